// Stochastic transport along rays: point density, ratio-tracking
// transmittance, weighted delta tracking, single / multiple scattering with
// fixed or per-segment stochastic masks (Sec. 3 radiative transfer; Sec. 4.5.1-
// 4.5.2 and Appendix B for the masks).
//
// Local majorant.  On a segment the tentative collisions form a Poisson
// process whose intensity is the masked envelope
//     mu(t) = sum_i rho m_c(i) |alpha_i| c_i exp(-M_i(x(t)) / 2) [M_i < r^2],
// an upper bound of |kappa| built only from primitives the segment crosses
// (m_c: majorant weight of cell c).  It is drawn as a superposition: on the
// chord [ci, co] of primitive i a homogeneous process of rate
// lambda_i = rho m |alpha_i| c_i exp(-h_i^2 / 2) (the envelope's maximum on
// the line) is thinned with probability exp(-n_i^2 (t - tc_i)^2 / 2), which
// leaves the chord's envelope as intensity.  One LBVH traversal proposes the
// points, a second one evaluates kappa and mu at all of them.
//
// Windows.  A lane holds at most a window's capacity of tentative points
// (TK, or fewer for the first windows of a segment that only seeks its
// first collision).  When a segment has more, the buffer keeps the earliest
// and the window ends at the last of them; the process is restarted just
// after it.  A Poisson process restarted at one of its own points (a
// stopping time) is again Poisson, so each window is an exact sample of the
// process restricted to it.
//
// Lanes.  A work unit is one sample of 64 rays, one ray per lane (all
// their samples, in groups of SG, where no per-sample storage is given).  Every
// lane of a wave runs the same steps (proposal traversal, evaluation
// traversal, decision) in each iteration of one flat loop, whatever its
// path length, so waves stay converged.  All random numbers of a sample come
// from counter-based streams keyed by (seed, ray, sample); a ray's result
// does not depend on the other rays of the launch.
#include <math.h>

#include "gf_hit.hpp"

#define TR_THREADS 64
#define TR_STACK 64  // deepest LBVH the per-lane traversal supports
#define TS_LDS 16    // per-lane stack entries kept in LDS; deeper ones go to the workspace
#define TK 64        // tentative points per window (also the bins of a CDF-inversion level)
#define CQ 6         // leaf candidates a lane queues before the wave processes them
#define DRAIN_LANES 4  // the wave drains its leaf queues once fewer lanes than this can step
#define SG 8         // samples whose secondary paths a lane follows back to back
// Cap of a cell's majorant multiplier.  The tentative points follow the
// envelope of the primitives scaled by min(cell weight, MAJ_CAP); where a
// weight exceeds the cap the envelope no longer bounds |kappa| of the
// reweighted field, which ratio tracking and the signed-weight delta
// tracking below tolerate (both are unbiased for any positive majorant):
// rare large weights (importance sampling of a badly aligned bin) then cost
// variance instead of an unbounded number of points.  18 is the largest
// weight of the uniform + control variate levels with the mixture bins.
#define MAJ_CAP 18.0f
// Hard bound on windows per segment (TK points each): a segment that would
// need more is cut short there, which keeps every wave's work finite.
#define MAX_WINDOWS 4096
// Waves resident in one launch: each owns a workspace slice, and loops over
// the launch's tiles with a grid stride.
#define TR_RES_BLOCKS 3072
// CDF inversion: levels of TK-bin refinement before the final linear step
#define FF_LEVELS 3

// Workspace rows of a wave (each row: TR_THREADS lanes x 4 B); the slice
// size is published to the other translation units as
// GF_TRACK_WAVE_FLOATS.  Rows [WS_KM, WS_KM + 2 TK) hold (kappa, mu) of the
// TK points as float2, point k of lane l at float2 index k TR_THREADS + l.
#define WS_KM 0
#define WS_XI (2 * TK)
#define WS_SPILL (3 * TK)
#define WS_TC (WS_SPILL + TR_STACK - TS_LDS)
#define WS_WF (WS_TC + SG)
#define WS_ROWS (WS_WF + SG)
static_assert(WS_ROWS * TR_THREADS == GF_TRACK_WAVE_FLOATS, "tracking slice size");

// sin and cos of 2 pi r for |r| <= 1/2 with the hardware's
// revolution-argument instructions: absolute error about 1.2e-7 on that
// range (measured against sincospif), for the estimators, whose errors
// are absolute; the optical-depth kernel keeps sincos_cycles, which stays
// relatively accurate near the zeros.
static __device__ __forceinline__ void sincos_rev(float r, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
}

// c_i / amp_i: the density's normalisation (2 pi)^-3/2 / (s0 s1 s2) over the
// optical-depth amplitude 1 / (4 pi s0 s1 s2), i.e. sqrt(2 / pi)
#define GF_NORM 0.79788456080286535588f

// Per-cell weights of the segment a lane is tracking: the density weight
// w_c of cell c sits in LDS (LaneMem::cw, one row per cell), its majorant
// multiplier is min(w_c, MAJ_CAP); `cells` holds the cells with a non-zero
// weight (they prune the traversal).
struct CellW {
    uint32_t cells;
};

static __device__ __forceinline__ CellW fixed_weights(uint32_t cells, float* wl) {
    CellW cw;
    cw.cells = cells & 0xFFFu;
#pragma unroll
    for (int c = 0; c < GF_NCELLS; ++c) wl[c * TR_THREADS] = ((cw.cells >> c) & 1u) ? 1.0f : 0.0f;
    return cw;
}

// Strategy of the per-segment stochastic masks (the Appendix B tables).
struct Strat {
    int level, bin;
    float beta, delta;
};

#define NLEV 4
#define NBIN 3

// x^e for x >= 0, e > 0 (exp / log intrinsics; x = 0 gives 0)
static __device__ __forceinline__ float pow_pos(float x, float e) { return x > 0.0f ? __expf(e * __logf(x)) : 0.0f; }

// Level weights (frequency-level table) for the uniform u: lw[l] of level l
// is `w0` for level 0 (the control variate), `wd` for the drawn level `ld`,
// and under accumulation 1 / (1 - (l/P)^e) for every level l <= ld.  With
// e = 1 - beta the power-law draw x = u^(1/e) falls in bucket [a, b) with
// probability b^e - a^e.
struct LevelDraw {
    int ld;
    float w0, wd;
    bool all, accum;
    float e;
    __device__ float weight(int l) const {
        if (all) return 1.0f;
        if (accum) return l <= ld ? 1.0f / (1.0f - pow_pos((float)l / NLEV, e)) : 0.0f;
        return l == ld ? wd : (l == 0 ? w0 : 0.0f);
    }
};

static __device__ __forceinline__ LevelDraw draw_level(const Strat& Z, float u) {
    LevelDraw D;
    D.e = 1.0f - Z.beta;
    D.all = Z.level == GF_LEVEL_ALL;
    D.accum = Z.level == GF_LEVEL_POWER_CV_ACCUM;
    D.w0 = 0.0f;
    D.ld = 0;
    D.wd = 0.0f;
    const float x = pow_pos(u, 1.0f / D.e);
    if (Z.level == GF_LEVEL_UNIFORM) {
        D.ld = min(NLEV - 1, (int)(NLEV * u));
        D.wd = (float)NLEV;
    } else if (Z.level == GF_LEVEL_POWER) {
        D.ld = min(NLEV - 1, (int)(NLEV * x));
        D.wd = 1.0f / (pow_pos((float)(D.ld + 1) / NLEV, D.e) - pow_pos((float)D.ld / NLEV, D.e));
    } else if (Z.level == GF_LEVEL_UNIFORM_CV) {
        D.w0 = 1.0f;
        D.ld = 1 + min(NLEV - 2, (int)((NLEV - 1) * u));
        D.wd = (float)(NLEV - 1);
    } else if (Z.level == GF_LEVEL_POWER_CV) {
        D.w0 = 1.0f;
        const int j = min(NLEV - 2, (int)((NLEV - 1) * x));
        D.ld = 1 + j;
        D.wd = 1.0f / (pow_pos((float)(j + 1) / (NLEV - 1), D.e) - pow_pos((float)j / (NLEV - 1), D.e));
    } else if (D.accum) {
        D.ld = min(NLEV - 1, (int)(NLEV * x));
    }
    return D;
}

// Bin weights (b0, b1, b2) of one level for the uniform u (orientation
// table); f_k the cell medians of |k_W| of the level, a_k the alignments
// |v.e_k| / |v|.
static __device__ __forceinline__ void bin_weights(const Strat& Z, float f0, float f1, float f2, float a0, float a1,
                                                   float a2, float u, float& b0, float& b1, float& b2) {
    b0 = b1 = b2 = 0.0f;
    if (Z.bin == GF_BIN_ALL) {
        b0 = b1 = b2 = 1.0f;
    } else if (Z.bin == GF_BIN_THRESHOLD) {
        b0 = a0 <= Z.delta ? 1.0f : 0.0f;
        b1 = a1 <= Z.delta ? 1.0f : 0.0f;
        b2 = a2 <= Z.delta ? 1.0f : 0.0f;
    } else if (Z.bin == GF_BIN_UNIFORM) {
        int k = min(NBIN - 1, (int)(NBIN * u));
        b0 = k == 0 ? (float)NBIN : 0.0f;
        b1 = k == 1 ? (float)NBIN : 0.0f;
        b2 = k == 2 ? (float)NBIN : 0.0f;
    } else if (Z.bin == GF_BIN_THRESHOLD_UNIFORM) {
        // bins within the threshold keep weight 1; one of the N others,
        // in axis order, is drawn with weight N
        const bool h0 = a0 > Z.delta, h1 = a1 > Z.delta, h2 = a2 > Z.delta;
        const int na = (int)h0 + (int)h1 + (int)h2;
        b0 = h0 ? 0.0f : 1.0f;
        b1 = h1 ? 0.0f : 1.0f;
        b2 = h2 ? 0.0f : 1.0f;
        if (na > 0) {
            const int j = min(na - 1, (int)(na * u));
            const int r0 = 0, r1 = (int)h0, r2 = (int)h0 + (int)h1;  // rank among the bins above
            if (h0 && r0 == j) b0 = (float)na;
            if (h1 && r1 == j) b1 = (float)na;
            if (h2 && r2 == j) b2 = (float)na;
        }
    } else {
        // importance (w_k / W) or its mixture with uniform; the log weights
        // are shifted by their maximum so that W >= 1 never underflows
        const float l0 = -0.5f * f0 * f0 * a0 * a0, l1 = -0.5f * f1 * f1 * a1 * a1, l2 = -0.5f * f2 * f2 * a2 * a2;
        const float mx = fmaxf(l0, fmaxf(l1, l2));
        const float w0 = __expf(l0 - mx), w1 = __expf(l1 - mx), w2 = __expf(l2 - mx);
        const float W = w0 + w1 + w2;
        float p0 = w0 / W, p1 = w1 / W, p2 = w2 / W;
        if (Z.bin == GF_BIN_MIXTURE) {
            p0 = 0.5f * p0 + 0.5f / NBIN;
            p1 = 0.5f * p1 + 0.5f / NBIN;
            p2 = 0.5f * p2 + 0.5f / NBIN;
        }
        // the bin whose cumulative range holds u; bins of probability 0 are
        // never drawn, and rounding past the sum falls to the last drawable
        int pick = -1;
        float acc = 0.0f;
        if (p0 > 0.0f) {
            pick = 0;
            acc += p0;
        }
        if (!(u < acc) && p1 > 0.0f) {
            pick = 1;
            acc += p1;
        }
        if (!(u < acc) && p2 > 0.0f) pick = 2;
        b0 = pick == 0 ? 1.0f / p0 : 0.0f;
        b1 = pick == 1 ? 1.0f / p1 : 0.0f;
        b2 = pick == 2 ? 1.0f / p2 : 0.0f;
    }
}

// A segment's stochastic cell weights (Sec. 4.5.1-4.5.2): four uniforms,
// u0 for the level strategy and u_l for the bins of each traced level
// l >= 1; level 0 keeps its bins with the level's weight.  Cells outside
// the fixed mask get weight 0.
static __device__ __forceinline__ CellW stochastic_weights(const SceneView& S, const Strat& Z, uint32_t fixed,
                                                           float vx, float vy, float vz, Rng& g, float* wl) {
    const float u0 = g.u(), u1 = g.u(), u2 = g.u(), u3 = g.u();
    const float vn = sqrtf(vx * vx + vy * vy + vz * vz);
    const float a0 = fabsf(vx) / vn, a1 = fabsf(vy) / vn, a2 = fabsf(vz) / vn;
    const LevelDraw D = draw_level(Z, u0);
    CellW cw;
    cw.cells = 0u;
#pragma unroll
    for (int l = 0; l < NLEV; ++l) {
        const float lw = D.weight(l);
        float b0 = 1.0f, b1 = 1.0f, b2 = 1.0f;
        if (l > 0 && lw != 0.0f)
            bin_weights(Z, S.med[NBIN * l], S.med[NBIN * l + 1], S.med[NBIN * l + 2], a0, a1, a2,
                        l == 1 ? u1 : (l == 2 ? u2 : u3), b0, b1, b2);
        const float w[NBIN] = {lw * b0, lw * b1, lw * b2};
#pragma unroll
        for (int k = 0; k < NBIN; ++k) {
            const int c = NBIN * l + k;
            const float wc = ((fixed >> c) & 1u) ? w[k] : 0.0f;
            wl[c * TR_THREADS] = wc;
            if (wc != 0.0f) cw.cells |= 1u << c;
        }
    }
    return cw;
}

// Work counters of the counting variants (per lane, summed at the end):
// accepted tentative points, internal nodes visited, primitive records read
// at leaves, windows.
struct Work {
    unsigned long long tent, nodes, prims, windows;
    unsigned long long used, pq_nodes, cover;  // points consumed; their point-query nodes and covers
};

// kappa at x under per-cell weights (rho alpha c exp(-M/2) cos(psi) summed)
template <bool COUNT>
static __device__ float point_density(const SceneView& S, const MaskView& M, float x, float y, float z,
                                      int* __restrict__ stk, Work& wk) {
    float acc = 0.0f;
    auto leaf = [&](int j) {
        PrimF P = load_prim(S.prims, j);
        if (COUNT) ++wk.prims;
        if (!mask_keep(M, P.cell, P.orig)) return;
        float dx = x - P.mux, dy = y - P.muy, dz = z - P.muz;
        float m = dx * (P.a00 * dx + P.a01 * dy + P.a02 * dz) + dy * (P.a01 * dx + P.a11 * dy + P.a12 * dz) +
                  dz * (P.a02 * dx + P.a12 * dy + P.a22 * dz);
        if (!(m < P.r2)) return;
        float ph = P.fx * dx + P.fy * dy + P.fz * dz + P.phi * (float)GF_INV_2PI;
        float s, c;
        sincos2pi(ph - rintf(ph), &s, &c);
        acc += P.amp * GF_NORM * __expf(-0.5f * m) * c;
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
        bool hl = (cells & 0xffffu & M.cells) && box_contains(nd->lbox, x, y, z);
        bool hr = ((cells >> 16) & M.cells) && box_contains(nd->rbox, x, y, z);
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
// per-lane memory: stack and tentative distances in LDS, the rest (point
// densities, majorants, delta-tracking uniforms, stack spill) in the
// launch's workspace, interleaved by lane so that a wave's rows coalesce
// ---------------------------------------------------------------------------
struct LaneMem {
    int* stk;   // LDS, TS_LDS entries, stride TR_THREADS
    int* cand;  // LDS, CQ queued leaf candidates, stride TR_THREADS
    float* t;   // LDS, TK tentative distances (or CDF bins), stride TR_THREADS
    float* cw;  // LDS, GF_NCELLS cell weights of the current segment, stride TR_THREADS
    float* ws;  // workspace: row r at ws[r * TR_THREADS]
    float2* km;  // workspace: (kappa, mu) of point k at km[k * TR_THREADS]
    __device__ float w(int c) const { return cw[c * TR_THREADS]; }
    __device__ float mw(int c) const { return fminf(cw[c * TR_THREADS], MAJ_CAP); }
    __device__ float2& kapmaj(int k) const { return km[k * TR_THREADS]; }
    __device__ float& xi(int k) const { return ws[(WS_XI + k) * TR_THREADS]; }
    __device__ float& ctc(int k) const { return ws[(WS_TC + k) * TR_THREADS]; }  // camera collision of sample k
    __device__ float& cwf(int k) const { return ws[(WS_WF + k) * TR_THREADS]; }  // its delta-tracking weight
    __device__ void push(int sp, int v) const {
        if (sp < TS_LDS)
            stk[sp * TR_THREADS] = v;
        else
            ((int*)ws)[(WS_SPILL + sp - TS_LDS) * TR_THREADS] = v;
    }
    __device__ int pop(int sp) const {
        return sp < TS_LDS ? stk[sp * TR_THREADS] : ((const int*)ws)[(WS_SPILL + sp - TS_LDS) * TR_THREADS];
    }
};

#define LANE_MEM(ws_base)                                                               \
    __shared__ int stk_all[TS_LDS * TR_THREADS];                                        \
    __shared__ int cand_all[CQ * TR_THREADS];                                           \
    __shared__ float t_all[TK * TR_THREADS];                                            \
    __shared__ float cw_all[GF_NCELLS * TR_THREADS];                                    \
    LaneMem lm;                                                                         \
    lm.stk = stk_all + threadIdx.x;                                                     \
    lm.cand = cand_all + threadIdx.x;                                                   \
    lm.t = t_all + threadIdx.x;                                                         \
    lm.cw = cw_all + threadIdx.x;                                                       \
    lm.ws = (ws_base) + (size_t)blockIdx.x * (WS_ROWS * TR_THREADS) + threadIdx.x;             \
    lm.km = (float2*)((ws_base) + (size_t)blockIdx.x * (WS_ROWS * TR_THREADS) + WS_KM * TR_THREADS) + threadIdx.x;

// chord of primitive P with the ray in float32: false when M < r^2 misses
// [ta, tb]; otherwise the clipped chord [ci, co], the closest-point parameter
// tc, n^2 = v.Av and h^2 (minimum of M on the line)
struct ChordF {
    float ci, co, tc, n2, h2;
};

static __device__ __forceinline__ bool chord_f32(const PrimF& P, float r2, float ox, float oy, float oz, float vx,
                                                 float vy, float vz, float ta, float tb, ChordF& C,
                                                 bool inclusive) {
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

// first point (ascending) at or after t
static __device__ __forceinline__ int first_point(const LaneMem& lm, int np, float t) {
    int lo = 0, hi = np;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (lm.t[mid * TR_THREADS] < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// entry distance of the ray into box b within [tmin, tmax] (INFINITY: miss);
// the same conservative test as slab_hit
static __device__ __forceinline__ float slab_enter(const float* b, float ox, float oy, float oz, float ix, float iy,
                                                   float iz, float tmin, float tmax) {
    float t0x = (b[0] - ox) * ix, t1x = (b[3] - ox) * ix;
    float t0y = (b[1] - oy) * iy, t1y = (b[4] - oy) * iy;
    float t0z = (b[2] - oz) * iz, t1z = (b[5] - oz) * iz;
    float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
    float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    return tn <= tf + fabsf(tf) * 1e-6f + 1e-30f ? tn : INFINITY;
}

// Per-lane front-to-back traversal of the nodes whose box meets [ta, tb]
// and whose subtree holds a weighted cell; leaf(j) for each such leaf.
// Leaves are not processed where they are found: a lane queues up to CQ of
// them, and once every lane's queue is full (or its traversal over) the wave
// processes the queues together, so the leaf work runs converged.  tb is
// re-read at every node, so a leaf callback may shrink it and prune what
// lies beyond.
template <bool COUNT, class LeafFn>
static __device__ __forceinline__ void lane_traverse(const SceneView& S, uint32_t cells, float ox, float oy, float oz,
                                                     float vx, float vy, float vz, float ta, const float& tb,
                                                     const LaneMem& lm, Work& wk, LeafFn&& leaf) {
    auto leaves = [&](int c) {
        int first, count;
        leaf_range(c, &first, &count);
        for (int k = 0; k < count; ++k) leaf(first + k);
    };
    if (S.croot < 0) {
        leaves(S.croot);
        return;
    }
    const float ix = 1.0f / vx, iy = 1.0f / vy, iz = 1.0f / vz;
    int sp = 0, node = 0, cnt = 0;
    bool trav = true;
    // one wave-uniform loop: a node step for every lane that still
    // traverses and has room in its queue; the queues are drained when fewer
    // than DRAIN_LANES lanes can step and some queue holds work (or when no
    // lane can step), so a few long traversals do not keep the rest of the
    // wave waiting on full queues.  A lane's leaves keep their order, so the
    // drain points do not change its result.
    for (;;) {
        bool step = trav && cnt <= CQ - 2;
        const unsigned long long bs = __ballot(step);
        if (bs == 0ull || (__popcll(bs) < DRAIN_LANES && __any(cnt > 0))) {
            for (int k = 0; k < cnt; ++k) leaves(lm.cand[k * TR_THREADS]);
            cnt = 0;
            if (!__any(trav)) break;
            continue;
        }
        if (!step) continue;
        const TNode* nd = S.cnodes + node;
        if (COUNT) ++wk.nodes;
        uint32_t c = nd->cells;
        float tbn = tb;
        float el = (c & 0xffffu & cells) ? slab_enter(nd->lbox, ox, oy, oz, ix, iy, iz, ta, tbn) : INFINITY;
        float er = ((c >> 16) & cells) ? slab_enter(nd->rbox, ox, oy, oz, ix, iy, iz, ta, tbn) : INFINITY;
        int lc = nd->lchild, rc = nd->rchild;
        if (el < INFINITY && lc < 0) {
            lm.cand[cnt * TR_THREADS] = lc;
            ++cnt;
            el = INFINITY;
        }
        if (er < INFINITY && rc < 0) {
            lm.cand[cnt * TR_THREADS] = rc;
            ++cnt;
            er = INFINITY;
        }
        if (el < INFINITY && er < INFINITY) {
            bool lfirst = el <= er;
            lm.push(sp, lfirst ? rc : lc);
            ++sp;
            node = lfirst ? lc : rc;
        } else if (el < INFINITY) {
            node = lc;
        } else if (er < INFINITY) {
            node = rc;
        } else if (sp == 0) {
            trav = false;
        } else {
            --sp;
            node = lm.pop(sp);
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

static __device__ __forceinline__ bool prim_on(const MaskView& M, int orig) {
    return !M.prim_bits || ((M.prim_bits[orig >> 5] >> (orig & 31)) & 1u);
}

// the largest tentative distance held (and its slot)
static __device__ __forceinline__ float latest_point(const LaneMem& lm, int np, int* slot) {
    float best = -INFINITY;
    int ks = 0;
    for (int k = 0; k < np; ++k) {
        float t = lm.t[k * TR_THREADS];
        if (t > best) {
            best = t;
            ks = k;
        }
    }
    *slot = ks;
    return best;
}

// One segment window [ta, tb] of the ray o + t v; lod2 the square of the
// continuous-LOD cutoff (0: off).
struct Seg {
    float ox, oy, oz, vx, vy, vz, ta, tb, lod2;
};

// Continuous LOD (supplementary "LOD Selection"): a primitive whose closest
// point lies at distance d = tc |v| ahead of the origin is left out when
// |f|^2 d^2 > lod_k^2 (its frequency is above the Nyquist limit there).
static __device__ __forceinline__ bool lod_drop(const PrimF& P, const Seg& sg, float tc) {
    if (!(sg.lod2 > 0.0f) || !(tc > 0.0f)) return false;
    float f2 = (P.fx * P.fx + P.fy * P.fy) + P.fz * P.fz;
    float v2 = sg.vx * sg.vx + sg.vy * sg.vy + sg.vz * sg.vz;
    return f2 * (tc * tc * v2) > sg.lod2;
}

// Proposal state of a window: points held, the window's capacity, and the
// window end (the segment end, or the last point held once the buffer is
// full, in slot `last`).
struct Prop {
    int np, cap, last;
    float tcut;
};

// Proposal work of one primitive P: draws its tentative points into lm.t /
// lm.xi.  The random numbers of a chord come from its own
// counter-based stream (segment key; primitive, window, proposal), so the
// points do not depend on the order in which chords are visited.
template <bool COUNT>
static __device__ void prop_leaf(const MaskView& M, const CellW& cw, const Seg& sg, uint32_t k0, uint32_t k1, int win,
                                 const PrimF& P, Prop& pr, const LaneMem& lm, Work& wk) {
    if (COUNT) ++wk.prims;
    float mw = lm.mw(P.cell);
    if (mw == 0.0f || !prim_on(M, P.orig)) return;
    ChordF C;
    if (!chord_f32(P, P.r2, sg.ox, sg.oy, sg.oz, sg.vx, sg.vy, sg.vz, sg.ta, pr.tcut, C, false)) return;
    if (lod_drop(P, sg, C.tc)) return;
    float lam = mw * fabsf(P.amp) * GF_NORM * __expf(-0.5f * C.h2);
    if (!(lam > 0.0f)) return;
    float inv = 1.0f / lam;
    float t = C.ci;
    for (uint32_t blk = 0;; ++blk) {
        uint4 r = philox4x32(make_uint4((uint32_t)P.orig, (uint32_t)win, blk, 0x50524f50u), k0, k1);
        // strict progress in float32 even when the gap rounds away
        t = fmaxf(t - __logf(unit_float(r.x)) * inv, nextafterf(t, INFINITY));
        if (!(t < fminf(C.co, pr.tcut))) break;
        float dt = t - C.tc;
        if (unit_float(r.y) >= __expf(-0.5f * C.n2 * dt * dt)) continue;  // thinning to the envelope
        float x = unit_float(r.z);
        if (COUNT) ++wk.tent;
        if (pr.np < pr.cap) {
            lm.t[pr.np * TR_THREADS] = t;
            lm.xi(pr.np) = x;
            ++pr.np;
            if (pr.np == pr.cap) pr.tcut = latest_point(lm, pr.np, &pr.last);
        } else {
            // full: the new point replaces the latest one
            lm.t[pr.last * TR_THREADS] = t;
            lm.xi(pr.last) = x;
            pr.tcut = latest_point(lm, pr.np, &pr.last);
        }
    }
}

// points in ascending order (the evaluation looks them up by bisection)
static __device__ void sort_points(const LaneMem& lm, int np) {
    for (int a = 1; a < np; ++a) {
        float tv = lm.t[a * TR_THREADS], xv = lm.xi(a);
        int b = a - 1;
        while (b >= 0 && lm.t[b * TR_THREADS] > tv) {
            lm.t[(b + 1) * TR_THREADS] = lm.t[b * TR_THREADS];
            lm.xi(b + 1) = lm.xi(b);
            --b;
        }
        lm.t[(b + 1) * TR_THREADS] = tv;
        lm.xi(b + 1) = xv;
    }
}

// kappa and mu contributions of primitive P (chord C) to the window's
// sorted points t[k0..] inside the chord.  kappa and mu take the same
// rounded envelope term, so kappa <= mu holds exactly where the carrier is 1
// (a positive density is then tracked with unit weights).
static __device__ __forceinline__ void add_chord(const PrimF& P, const ChordF& C, const CellW& cw, float mw,
                                                 const Seg& sg, int np, int k, const LaneMem& lm) {
    float am = P.amp * GF_NORM, aa = fabsf(am);
    float ws = copysignf(lm.w(P.cell), am);
    // carrier phase (cycles) along the chord: its value at the closest
    // point plus its slope times the distance from there
    const float yx = sg.ox + C.tc * sg.vx - P.mux, yy = sg.oy + C.tc * sg.vy - P.muy,
                yz = sg.oz + C.tc * sg.vz - P.muz;
    const float thc = P.fx * yx + P.fy * yy + P.fz * yz + P.phi * (float)GF_INV_2PI;
    const float dph = P.fx * sg.vx + P.fy * sg.vy + P.fz * sg.vz;
    for (; k < np; ++k) {
        float t = lm.t[k * TR_THREADS];
        if (t > C.co) break;
        float dt = t - C.tc;
        float e = __expf(-0.5f * (C.h2 + C.n2 * dt * dt));
        float ph = fmaf(dt, dph, thc);
        float sn, cs;
        sincos_rev(ph - rintf(ph), &sn, &cs);
        float ce = aa * e;
        float2 v = lm.kapmaj(k);
        v.x += ws * (ce * cs);
        v.y += mw * ce;
        lm.kapmaj(k) = v;
    }
}


// Evaluation pass of a lane's own window: kappa (density weights) and mu
// (majorant weights) at its np sorted points, from every chord that contains
// them (a second per-lane traversal over [first point, last point]).
template <bool COUNT>
static __device__ void evaluate(const SceneView& S, const MaskView& M, const CellW& cw, const Seg& sg, int np,
                                const LaneMem& lm, Work& wk) {
    const float pa = lm.t[0], pb = lm.t[(np - 1) * TR_THREADS];
    lane_traverse<COUNT>(S, cw.cells, sg.ox, sg.oy, sg.oz, sg.vx, sg.vy, sg.vz, pa, pb, lm, wk, [&](int j) {
        PrimF P = load_prim(S.prims, j);
        if (COUNT) ++wk.prims;
        float mw = lm.mw(P.cell);
        if (mw == 0.0f || !prim_on(M, P.orig)) return;
        ChordF C;
        if (!chord_f32(P, P.r2, sg.ox, sg.oy, sg.oz, sg.vx, sg.vy, sg.vz, pa, pb, C, true)) return;
        if (lod_drop(P, sg, C.tc)) return;
        add_chord(P, C, cw, mw, sg, np, first_point(lm, np, C.ci), lm);
    });
}

// Signed-weight delta tracking at one tentative point: real with probability
// |kappa| / (|kappa| + |mu - kappa|), weight factor sign(kappa) D / mu on a
// real collision and sign(mu - kappa) D / mu on a null one (D the sum of the
// two magnitudes).  Woodcock tracking, with unit factors, when 0 <= kappa <= mu.
static __device__ __forceinline__ bool delta_real(float kap, float mu, float xi, float* fac_real, float* fac_null) {
    if (kap >= 0.0f && kap <= mu) {
        *fac_real = *fac_null = 1.0f;
        return xi * mu < kap;
    }
    float kn = mu - kap, D = fabsf(kap) + fabsf(kn);
    *fac_real = copysignf(D / mu, kap);
    *fac_null = copysignf(D / mu, kn);
    return xi * D < fabsf(kap);
}

#define MODE_RATIO 1
#define MODE_DELTA 2

// State of the segment a lane is tracking.
struct SegState {
    Seg sg;
    CellW cw;
    int mode, win;
    bool live;    // window left to track
    float T;      // ratio-tracking product (exact: exp(-tau) of the segment)
    float wf;     // delta-tracking weight factor
    float tc;     // collision distance (INFINITY: none)
    float fs;     // CDF inversion: the optical depth -log(1 - xi) to reach
    uint32_t k0, k1;  // key of the segment's chord streams
};

static __device__ __forceinline__ void begin_segment(const SceneView& S, SegState& st, const float* o,
                                                     const float* v, float t0, float t1, const CellW& cw, int mode,
                                                     float lod2, Rng& g) {
    st.k0 = g.bits();
    st.k1 = g.bits();
    st.sg.ox = o[0];
    st.sg.oy = o[1];
    st.sg.oz = o[2];
    st.sg.vx = v[0];
    st.sg.vy = v[1];
    st.sg.vz = v[2];
    st.sg.ta = t0;
    st.sg.tb = t1;
    st.sg.lod2 = lod2;
    st.live = clip_box(S, o[0], o[1], o[2], v[0], v[1], v[2], st.sg.ta, st.sg.tb);
    st.cw = cw;
    st.mode = mode;
    st.win = 0;
    st.T = 1.0f;
    st.wf = 1.0f;
    st.tc = INFINITY;
    st.fs = 0.0f;
}

// CDF inversion: the optical depth s = -log(1 - xi) at which the segment's
// free flight ends
static __device__ __forceinline__ void draw_flight(SegState& st, Rng& g) { st.fs = -__logf(1.0f - g.u()); }

// Capacity of the next window of a segment.  A segment tracked for its
// first real collision only (delta tracking without a transmittance
// estimate) uses the points of a window up to that collision and drops the
// rest, so its windows start at WIN0 points and double up to TK; a segment
// whose ratio-tracking estimate consumes every point takes TK at once.
// Windows of any capacity are exact samples (the window ends at one of the
// process's own points).
#define WIN0 8
static __device__ __forceinline__ int window_cap(const SegState& st) {
    return st.mode == MODE_DELTA ? min(TK, WIN0 << min(st.win, 3)) : TK;
}

static __device__ __forceinline__ void begin_prop(Prop& pr, const SegState& st) {
    pr.np = 0;
    pr.cap = window_cap(st);
    pr.last = 0;
    pr.tcut = st.sg.tb;
}

// Proposal pass of a lane's own window: per-lane LBVH traversal (incoherent
// secondary rays).
template <bool COUNT>
static __device__ void lane_propose(const SceneView& S, const MaskView& M, const SegState& st, Prop& pr,
                                    const LaneMem& lm, Work& wk) {
    const Seg& sg = st.sg;
    lane_traverse<COUNT>(S, st.cw.cells, sg.ox, sg.oy, sg.oz, sg.vx, sg.vy, sg.vz, sg.ta, pr.tcut, lm, wk,
                         [&](int j) {
                             prop_leaf<COUNT>(M, st.cw, sg, st.k0, st.k1, st.win, load_prim(S.prims, j), pr, lm, wk);
                         });
}

// Packet traversal for the windows of a whole wave at once (coherent camera
// rays): the node index, the stack (LDS, pstk) and the leaf are
// wave-uniform, so node records come through the scalar cache; each lane
// tests its own ray over its own [ta, tb] (tb re-read at every node) and the
// wave descends where any lane hits; leaf(j, record of j) runs on the lanes
// whose ray meets the leaf's box.  Children are visited left first, so the leaves a
// lane processes come in tree order whatever the other lanes do.
template <bool COUNT, bool PF, class LeafFn>
static __device__ __forceinline__ void packet_walk(const SceneView& S, const SegState& st, bool act, float ta,
                                                   const float& tb, int* __restrict__ pstk, Work& wk, LeafFn&& leaf) {
    const Seg& sg = st.sg;
    // a leaf's records are wave-uniform scalar loads; the next one is
    // issued before the current one is processed, so its latency overlaps
    // that work
    auto leaves = [&](int c) {
        int first, count;
        leaf_range(c, &first, &count);
        PrimF nx = load_prim(S.prims, first);
        for (int k = 0; k < count; ++k) {
            const PrimF P = nx;
            if (k + 1 < count) nx = load_prim(S.prims, first + k + 1);
            leaf(first + k, P);
        }
    };
    if (S.croot < 0) {
        if (act) leaves(S.croot);
        return;
    }
    const float ix = 1.0f / sg.vx, iy = 1.0f / sg.vy, iz = 1.0f / sg.vz;
    int sp = 0;
    TNode cur = S.cnodes[0];
    for (;;) {
        if (COUNT && act) ++wk.nodes;
        const int lc = cur.lchild, rc = cur.rchild;
        // PF: the internal children's records are loaded before this node's
        // tests and leaves, so a step down finds them in registers (32 more
        // scalar registers; only the instance that has them to spare asks)
        TNode nl, nr;
        if (PF) {
            if (lc >= 0) nl = S.cnodes[lc];
            if (rc >= 0) nr = S.cnodes[rc];
        }
        const uint32_t c = cur.cells;
        float tbn = tb;
        bool hl = act && (c & 0xffffu & st.cw.cells) && slab_hit(cur.lbox, sg.ox, sg.oy, sg.oz, ix, iy, iz, ta, tbn);
        bool hr = act && ((c >> 16) & st.cw.cells) && slab_hit(cur.rbox, sg.ox, sg.oy, sg.oz, ix, iy, iz, ta, tbn);
        uint64_t bl = __ballot(hl), br = __ballot(hr);
        if (bl && lc < 0) {
            if (hl) leaves(lc);
            bl = 0;
        }
        if (br && rc < 0) {
            if (hr) leaves(rc);
            br = 0;
        }
        if (bl && br) {
            pstk[sp] = rc;
            ++sp;
            cur = PF ? nl : S.cnodes[lc];
        } else if (bl) {
            cur = PF ? nl : S.cnodes[lc];
        } else if (br) {
            cur = PF ? nr : S.cnodes[rc];
        } else {
            if (sp == 0) break;
            --sp;
            cur = S.cnodes[uniform_int(pstk[sp])];
        }
    }
}

// kappa and mu from primitive P at the sorted points of a window in [pa, pb]
template <bool COUNT>
static __device__ __forceinline__ void eval_leaf(const MaskView& M, const SegState& st, const PrimF& P, float pa,
                                                 float pb, int np, const LaneMem& lm, Work& wk) {
    if (COUNT) ++wk.prims;
    float mw = lm.mw(P.cell);
    if (mw == 0.0f || !prim_on(M, P.orig)) return;
    ChordF C;
    if (!chord_f32(P, P.r2, st.sg.ox, st.sg.oy, st.sg.oz, st.sg.vx, st.sg.vy, st.sg.vz, pa, pb, C, true)) return;
    if (lod_drop(P, st.sg, C.tc)) return;
    add_chord(P, C, st.cw, mw, st.sg, np, first_point(lm, np, C.ci), lm);
}

// points sorted, kappa and mu cleared: ready for an evaluation pass
static __device__ __forceinline__ void open_points(const LaneMem& lm, int np) {
    sort_points(lm, np);
    for (int k = 0; k < np; ++k) lm.kapmaj(k) = make_float2(0.0f, 0.0f);
}

// Decisions of an evaluated window and the move to the next one.  Returns
// true when the segment is finished.
// Work of a point query at x, the unit of the algorithmic bytes of tracking:
// internal nodes whose box contains x on the walk from the root (pruned by
// the cells), and primitives of weighted cells whose truncated support
// contains x.  Counting variants only.
static __device__ void count_point_query(const SceneView& S, const MaskView& M, uint32_t cells, const LaneMem& lm,
                                         float x, float y, float z, Work& wk) {
    auto leaf = [&](int j) {
        PrimF P = load_prim(S.prims, j);
        if (!((cells >> P.cell) & 1u) || !prim_on(M, P.orig)) return;
        float dx = x - P.mux, dy = y - P.muy, dz = z - P.muz;
        float m = dx * (P.a00 * dx + P.a01 * dy + P.a02 * dz) + dy * (P.a01 * dx + P.a11 * dy + P.a12 * dz) +
                  dz * (P.a02 * dx + P.a12 * dy + P.a22 * dz);
        if (m < P.r2) ++wk.cover;
    };
    if (S.n == 1) {
        leaf(0);
        return;
    }
    int sp = 0, node = 0;
    for (;;) {
        const TNode* nd = S.nodes + node;
        ++wk.pq_nodes;
        uint32_t c = nd->cells;
        bool hl = (c & 0xffffu & cells) && box_contains(nd->lbox, x, y, z);
        bool hr = ((c >> 16) & cells) && box_contains(nd->rbox, x, y, z);
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
            lm.push(sp, rc);
            ++sp;
            node = lc;
        } else if (hl) {
            node = lc;
        } else if (hr) {
            node = rc;
        } else {
            if (sp == 0) break;
            --sp;
            node = lm.pop(sp);
        }
    }
}

template <bool COUNT>
static __device__ bool decide_window(const SceneView& S, const MaskView& M, SegState& st, const Prop& pr,
                                     const LaneMem& lm, Work& wk) {
    if (!st.live) return true;
    if (COUNT) ++wk.windows;
    const int np = pr.np;
    if (COUNT) {
        // the points the estimators consume: all of them for ratio
        // tracking, up to the collision for delta tracking
        int used = np;
        if (!(st.mode & MODE_RATIO) && (st.mode & MODE_DELTA) && !(st.tc < INFINITY)) {
            float fr, fn;
            for (int k = 0; k < np; ++k) {
                const float2 v = lm.kapmaj(k);
                if (delta_real(v.x, v.y, lm.xi(k), &fr, &fn)) {
                    used = k + 1;
                    break;
                }
            }
        }
        wk.used += used;
        for (int k = 0; k < used; ++k) {
            const float t = lm.t[k * TR_THREADS];
            count_point_query(S, M, st.cw.cells, lm, st.sg.ox + t * st.sg.vx, st.sg.oy + t * st.sg.vy,
                              st.sg.oz + t * st.sg.vz, wk);
        }
    }
    if (st.mode & MODE_RATIO)
        for (int k = 0; k < np; ++k) {
            const float2 v = lm.kapmaj(k);
            st.T *= 1.0f - v.x / v.y;
        }
    if ((st.mode & MODE_DELTA) && !(st.tc < INFINITY)) {
        // the collision is the earliest real point; null factors of the
        // points before it apply
        float w = 1.0f, fr, fn;
        for (int k = 0; k < np; ++k) {
            const float2 v = lm.kapmaj(k);
            bool real = delta_real(v.x, v.y, lm.xi(k), &fr, &fn);
            if (real) {
                w *= fr;
                st.tc = lm.t[k * TR_THREADS];
                break;
            }
            w *= fn;
        }
        st.wf *= w;
    }
    bool full = pr.tcut < st.sg.tb;
    bool stop = !full || (st.mode == MODE_DELTA && st.tc < INFINITY) || ++st.win >= MAX_WINDOWS;
    if (!stop) st.sg.ta = pr.tcut;
    return stop;
}

// A lane's own window after its proposal pass: evaluation and decisions.
template <bool COUNT>
static __device__ bool close_window(const SceneView& S, const MaskView& M, SegState& st, const Prop& pr,
                                    const LaneMem& lm, Work& wk) {
    if (st.live && pr.np > 0) {
        open_points(lm, pr.np);
        evaluate<COUNT>(S, M, st.cw, st.sg, pr.np, lm, wk);
    }
    return decide_window<COUNT>(S, M, st, pr, lm, wk);
}

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

// Order in which a launch hands out the chunks of an image: first the
// central half of the columns of 8x8 tiles, then the outer columns, each
// part by rows from the middle of the image outward (middle row, the one
// above, the one below, ...), so the dense centre, whose chunks take
// longest, starts first and the launch does not end on a few slow chunks.
// A bijection on the chunk indices; a ray's result does not depend on when
// it is traced.
static __device__ __forceinline__ int tile_order(int c, int nchunks, int tile_w) {
    if (tile_w <= 0) return c;
    const int tiles_x = tile_w >> 3, tiles_y = nchunks / tiles_x;
    const int x0 = tiles_x >> 2, wa = tiles_x - 2 * x0, na = wa * tiles_y;
    int q, tx;
    if (c < na) {
        q = c / wa;
        tx = x0 + (c - q * wa);
    } else {
        const int wb = tiles_x - wa, c2 = c - na;
        q = c2 / wb;
        const int r = c2 - q * wb;
        tx = r < x0 ? r : r + wa;
    }
    const int mid = tiles_y >> 1;
    const int ty = (q & 1) ? mid - ((q + 1) >> 1) : mid + (q >> 1);
    return ty * tiles_x + tx;
}

static int64_t tr_threads(int64_t n, int tile_w) {
    if (tile_w <= 0) return n;
    return (int64_t)(tile_w / 8) * ((n / tile_w + 7) / 8) * 64;
}

// ---------------------------------------------------------------------------
// per-ray drivers
// ---------------------------------------------------------------------------
struct RenderArgs {
    int spp, multiple, max_scatter, stochastic, exact;
    float albedo, hg, env;
    Strat strat;
    uint32_t shadow_cells;  // 0: shadow segments draw their own mask
    int tile_w;             // image width of the launch's 8x8 tiles (0: a ray list)
    int su, groups;         // samples per work unit; units per chunk of 64 rays (groups * su >= spp)
    int n;                  // rays of the launch (of the request, when serving)
    float* part;            // split samples: per-sample L (spp x n), then per-sample T (spp x n) if keep_T; else NULL
    int keep_T;
    uint64_t seed;
};

// Running sums of a ray's samples (radiance L and primary transmittance T)
// and the mean / variance taken from them.  The render lanes and the
// reduction of per-sample values use this one accumulation, in sample order,
// so a ray's result has the same bits whichever way its samples were split
// into work units.
struct SampleSums {
    float s1, s2, q1, q2;
    __device__ void zero() { s1 = s2 = q1 = q2 = 0.0f; }
    __device__ void add_L(float x) {
        s1 += x;
        s2 = fmaf(x, x, s2);
    }
    __device__ void add_T(float x) {
        q1 += x;
        q2 = fmaf(x, x, q2);
    }
    // sample variance; +inf when the sums overflowed float32 (a heavy tail
    // of the signed delta-tracking weights), never a silent 0
    static __device__ float variance(float a1, float a2, float inv, int n) {
        if (n < 2) return 0.0f;
        float v = (a2 - a1 * a1 * inv) / (n - 1);
        return v >= 0.0f ? v : (v < 0.0f ? 0.0f : INFINITY);
    }
    __device__ void result(int spp, float* out4) const {
        float inv = 1.0f / spp;
        out4[0] = s1 * inv;
        out4[1] = variance(s1, s2, inv, spp);
        out4[2] = q1 * inv;
        out4[3] = variance(q1, q2, inv, spp);
    }
};

// ---------------------------------------------------------------------------
// Free flights by CDF inversion (Sec. 3: a collision at x_t solves
// log(1 - xi) = -sum_i tau_i(x_0, x_t); Sec. 4.4, distance sampling by
// inverting the closed-form optical depth) and exact transmittance.
// The optical depth over [lo, hi] is split into TK bins of equal length:
// every crossed chord adds its closed-form integral over each bin piece it
// covers (the segment integral of Sec. 4.4 with the piece's ends as bounds,
// binary64 chord geometry).  The bins give the segment's optical depth
// (T = exp(-tau)) and the first bin where the cumulative depth reaches
// s = -log(1 - xi); FF_LEVELS rounds of splitting that bin into TK sub-bins
// narrow the collision to (hi - lo) / TK^FF_LEVELS, inside which the depth
// is taken as linear.  The path escapes when the depth of the whole segment
// is below s.  For a non-negative density the distance follows
// 1 - exp(-tau(ta, t)) up to that last linear step; where the mixture is
// negative the cumulative depth need not be monotone and the sampler returns
// its first crossing.  The bins reuse the lane's tentative-point row.
// ---------------------------------------------------------------------------
__constant__ float c_weid_tr[WEID_N];
__constant__ float c_weidL_tr;
__constant__ double c_weid64_tr[WEID64_N];
__constant__ double c_weidL64_tr;

static bool g_weid_tr_ready[64];

gf_status gf_ensure_weideman_track() {
    int dev = 0;
    GF_HIP(hipGetDevice(&dev));
    if (dev >= 0 && dev < 64 && g_weid_tr_ready[dev]) return GF_OK;
    float a[WEID_N], L;
    gf_weideman_coeffs(a, &L);
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weid_tr), a, sizeof(a)));
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weidL_tr), &L, sizeof(L)));
    double a64[WEID64_N], L64;
    gf_weideman_coeffs64(a64, &L64);
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weid64_tr), a64, sizeof(a64)));
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weidL64_tr), &L64, sizeof(L64)));
    if (dev >= 0 && dev < 64) g_weid_tr_ready[dev] = true;
    return GF_OK;
}

// Weighted optical depth of primitive j's chord over [lo, hi], added to the
// TK bins of width (hi - lo) / TK piece by piece.
template <bool COUNT>
static __device__ void bin_chord(const SceneView& S, const MaskView& M, const SegState& st, int j, const PrimF& P,
                                 float lo, float hi, const LaneMem& lm, Work& wk) {
    if (COUNT) ++wk.prims;
    const float w = lm.w(P.cell);
    if (w == 0.0f || !prim_on(M, P.orig)) return;
    RayD R;
    R.ox = st.sg.ox; R.oy = st.sg.oy; R.oz = st.sg.oz;
    R.vx = st.sg.vx; R.vy = st.sg.vy; R.vz = st.sg.vz;
    R.tmin = lo; R.tmax = hi;
    HitGeom H;
    if (!hit_geom(P, R, S.A64 + (size_t)j * GF_A64, H)) return;
    if (lod_drop(P, st.sg, (float)H.tc)) return;
    const double dlo = lo, dw = ((double)hi - dlo) / TK;
    const double ta = H.tc + H.uad * H.inv_n, tb = H.tc + H.ubd * H.inv_n;
    const int b0 = min(TK - 1, max(0, (int)floor((ta - dlo) / dw)));
    const int b1 = min(TK - 1, max(0, (int)floor((tb - dlo) / dw)));
    for (int b = b0; b <= b1; ++b) {
        double p0 = fmax(ta, dlo + b * dw), p1 = fmin(tb, dlo + (b + 1) * dw);
        if (!(p0 < p1)) continue;
        HitGeom Hp = H;
        Hp.enda = H.enda && b == b0;
        Hp.endb = H.endb && b == b1;
        Hp.uad = Hp.enda ? -H.halfd : H.n * (p0 - H.tc);
        Hp.ubd = Hp.endb ? H.halfd : H.n * (p1 - H.tc);
        Hp.ua = (float)Hp.uad;
        Hp.ub = (float)Hp.ubd;
        lm.t[b * TR_THREADS] += w * hit_value(P, Hp, c_weid_tr, c_weidL_tr, c_weid64_tr, c_weidL64_tr);
    }
}

// One binning pass over each active lane's [lo, hi]: a packet walk (camera
// segments) or per-lane traversals (secondary segments).
template <bool COUNT, bool PACKET>
static __device__ void bin_pass(const SceneView& S, const MaskView& M, const SegState& st, bool act, float lo,
                                float hi, const LaneMem& lm, int* pstk, Work& wk) {
    if (act)
        for (int b = 0; b < TK; ++b) lm.t[b * TR_THREADS] = 0.0f;
    auto leaf = [&](int j, const PrimF& P) { bin_chord<COUNT>(S, M, st, j, P, lo, hi, lm, wk); };
    if (PACKET) {
        packet_walk<COUNT, false>(S, st, act, lo, hi, pstk, wk, leaf);
    } else if (act) {
        const Seg& sg = st.sg;
        lane_traverse<COUNT>(S, st.cw.cells, sg.ox, sg.oy, sg.oz, sg.vx, sg.vy, sg.vz, lo, hi, lm, wk,
                             [&](int j) { leaf(j, load_prim(S.prims, j)); });
    }
}

// Exact transmittance and (MODE_DELTA) the CDF-inversion collision of the
// segments of the active lanes; every lane of the wave calls it.
template <bool COUNT, bool PACKET>
static __device__ void exact_segment(const SceneView& S, const MaskView& M, SegState& st, bool act, const LaneMem& lm,
                                     int* pstk, Work& wk) {
    act = act && st.live;
    float lo = st.sg.ta, hi = st.sg.tb, acc = 0.0f, frac = 0.0f;
    bool seek = act && (st.mode & MODE_DELTA);
    for (int lev = 0; lev < FF_LEVELS; ++lev) {
        // only lanes still searching (and, first, every active lane) bin
        const bool bin = lev == 0 ? act : seek;
        if (PACKET ? !__any(bin) : !bin) break;
        bin_pass<COUNT, PACKET>(S, M, st, bin, lo, hi, lm, pstk, wk);
        if (lev == 0 && act) {
            float tot = 0.0f;
            for (int b = 0; b < TK; ++b) tot += lm.t[b * TR_THREADS];
            st.T = __expf(-tot);
            if (!(tot >= st.fs)) seek = false;  // escape
        }
        if (seek) {
            // first bin whose cumulative depth reaches s (the last bin when
            // rounding leaves the sub-bins' sum just below their parent's)
            int b = TK - 1;
            float d = lm.t[b * TR_THREADS];
            for (int k = 0; k < TK; ++k) {
                float dk = lm.t[k * TR_THREADS];
                if (acc + dk >= st.fs || k == TK - 1) {
                    b = k;
                    d = dk;
                    break;
                }
                acc += dk;
            }
            frac = d > 0.0f ? fminf(1.0f, fmaxf(0.0f, (st.fs - acc) / d)) : 0.5f;
            const float dw = (hi - lo) / TK;
            lo = lo + b * dw;
            hi = lo + dw;
        }
    }
    if (seek) st.tc = lo + frac * (hi - lo);
    if (act) st.live = false;
}

// e^{-u^2/2} Re{e^{i psi(u)} w((sgn(u) Omega + i|u|)/sqrt 2)} in float32
// (psi(u) = 2 pi (thc + u omc), phases in cycles)
static __device__ __forceinline__ float tail_f32(float u, float Om, float thc, float omc) {
    const float is2 = 0.70710678118654752440f;
    const float sg = u < 0.0f ? -1.0f : 1.0f;
    const float2 w = wofz_weideman(sg * Om * is2, fabsf(u) * is2, c_weid_tr, c_weidL_tr);
    const float c = fmaf(u, omc, thc);
    float sp, cp;
    sincos_rev(c - rintf(c), &sp, &cp);
    return __expf(-0.5f * u * u) * (cp * w.x - sp * w.y);
}

// Optical depth of primitive P over [ta, tb] of segment sg for the render's
// closed-form transmittance exp(-sum): the segment integral of Sec. 4.4
// (Re{e^{i theta} [E(u_b) - E(u_a)]}, Appendix A) with float32 chord
// geometry and float32 Faddeeva evaluations, one branch-free form for every
// hit.  Where the difference cancels (short or strongly oscillating chords)
// its error stays near float32 rounding of the terms, an absolute error of
// about 1e-7 of the primitive's peak contribution, far below the Monte Carlo
// error of the radiance it enters; the optical-depth kernel keeps its
// binary64 geometry, quadrature and binary64 fallbacks for its relative
// bound.  False when the chord is empty; *tc: closest-point parameter.
static __device__ __forceinline__ bool shadow_tau_f32(const PrimF& P, const Seg& sg, float ta, float tb, float* tau,
                                                      float* tc_out) {
    const float dx = sg.ox - P.mux, dy = sg.oy - P.muy, dz = sg.oz - P.muz;
    const float avx = P.a00 * sg.vx + P.a01 * sg.vy + P.a02 * sg.vz;
    const float avy = P.a01 * sg.vx + P.a11 * sg.vy + P.a12 * sg.vz;
    const float avz = P.a02 * sg.vx + P.a12 * sg.vy + P.a22 * sg.vz;
    const float a = sg.vx * avx + sg.vy * avy + sg.vz * avz;
    const float tc = -(dx * avx + dy * avy + dz * avz) / a;
    const float yx = dx + tc * sg.vx, yy = dy + tc * sg.vy, yz = dz + tc * sg.vz;
    const float h2 = yx * (P.a00 * yx + P.a01 * yy + P.a02 * yz) + yy * (P.a01 * yx + P.a11 * yy + P.a12 * yz) +
                     yz * (P.a02 * yx + P.a12 * yy + P.a22 * yz);
    if (!(h2 < P.r2)) return false;
    const float n = sqrtf(a), inv_n = 1.0f / n;
    const float half = sqrtf(P.r2 - h2), hn = half * inv_n;
    const float tin = tc - hn, tout = tc + hn;
    const float lo = fmaxf(ta, tin), hi = fminf(tb, tout);
    if (!(lo < hi)) return false;
    const bool enda = !(ta > tin), endb = !(tb < tout);
    const float thc = P.fx * yx + P.fy * yy + P.fz * yz + P.phi * (float)GF_INV_2PI;
    const float omc = (P.fx * sg.vx + P.fy * sg.vy + P.fz * sg.vz) * inv_n;
    const float Om = 2.0f * (float)GF_PI * omc;
    const float eO = __expf(-0.5f * Om * Om);
    float sth, cth;
    sincos_rev(thc - rintf(thc), &sth, &cth);
    float val;
    if (enda && endb) {
        // the whole chord: E(h) - E(-h) = 2 Re E(h)
        val = 2.0f * cth * (eO - tail_f32(half, Om, 0.0f, omc));
    } else {
        const float ua = enda ? -half : n * (lo - tc), ub = endb ? half : n * (hi - tc);
        const float sa = ua < 0.0f ? -1.0f : 1.0f, sb = ub < 0.0f ? -1.0f : 1.0f;
        val = (sb - sa) * eO * cth - sb * tail_f32(ub, Om, thc, omc) + sa * tail_f32(ua, Om, thc, omc);
    }
    *tau = P.amp * inv_n * __expf(-0.5f * h2) * val;
    *tc_out = tc;
    return true;
}

// Closed-form transmittance exp(-tau) of a lane's own segment: one
// traversal summing the closed-form integrals of the crossed chords
// (Sec. 4.4, float32: shadow_tau_f32), the way the tomography case of
// Sec. 4.6 turns optical depth into transmittance.  Its mean equals that of
// ratio tracking, with no variance.
template <bool COUNT>
static __device__ void exact_T_own(const SceneView& S, const MaskView& M, SegState& st, const LaneMem& lm, Work& wk) {
    if (!st.live) return;
    float acc = 0.0f;
    const Seg& sg = st.sg;
    lane_traverse<COUNT>(S, st.cw.cells, sg.ox, sg.oy, sg.oz, sg.vx, sg.vy, sg.vz, sg.ta, sg.tb, lm, wk, [&](int j) {
        PrimF P = load_prim(S.prims, j);
        if (COUNT) ++wk.prims;
        const float w = lm.w(P.cell);
        if (w == 0.0f || !prim_on(M, P.orig)) return;
        float tau, tc;
        if (!shadow_tau_f32(P, sg, sg.ta, sg.tb, &tau, &tc)) return;
        if (lod_drop(P, sg, tc)) return;
        acc += w * tau;
    });
    st.T = __expf(-acc);
    st.live = false;
}

// Closed-form transmittance of the segments of a whole wave in one packet walk
// (the rays of a tile's shadow segments share their direction, so the
// packet stays coherent); every lane of the wave calls it.
template <bool COUNT>
static __device__ void exact_T_packet(const SceneView& S, const MaskView& M, SegState& st, bool act, const LaneMem& lm,
                                      int* pstk, Work& wk) {
    act = act && st.live;
    float acc = 0.0f;
    packet_walk<COUNT, true>(S, st, act, st.sg.ta, st.sg.tb, pstk, wk, [&](int, const PrimF& P) {
        if (COUNT) ++wk.prims;
        const float w = lm.w(P.cell);
        if (w == 0.0f || !prim_on(M, P.orig)) return;
        float tau, tc;
        if (!shadow_tau_f32(P, st.sg, st.sg.ta, st.sg.tb, &tau, &tc)) return;
        if (lod_drop(P, st.sg, tc)) return;
        acc += w * tau;
    });
    if (act) {
        st.T = __expf(-acc);
        st.live = false;
    }
}

// Camera segments of a whole wave, window by window: packet proposal and
// packet evaluation passes; a lane whose segment is finished sits out.
template <bool COUNT, bool PF>
static __device__ void track_camera(const SceneView& S, const MaskView& M, SegState& st, bool valid,
                                    const LaneMem& lm, int* pstk, Work& wk) {
    bool open = valid && st.live;
    while (__any(open)) {
        Prop pr;
        begin_prop(pr, st);
        packet_walk<COUNT, PF>(S, st, open, st.sg.ta, pr.tcut, pstk, wk, [&](int, const PrimF& P) {
            prop_leaf<COUNT>(M, st.cw, st.sg, st.k0, st.k1, st.win, P, pr, lm, wk);
        });
        const bool ev = open && pr.np > 0;
        if (ev) open_points(lm, pr.np);
        const float pa = ev ? lm.t[0] : 0.0f, pb = ev ? lm.t[(pr.np - 1) * TR_THREADS] : -1.0f;
        packet_walk<COUNT, PF>(S, st, ev, pa, pb, pstk, wk,
                           [&](int, const PrimF& P) { eval_leaf<COUNT>(M, st, P, pa, pb, pr.np, lm, wk); });
        if (open && decide_window<COUNT>(S, M, st, pr, lm, wk)) open = false;
    }
}

// A lane's own (secondary) segment, one window; true when it is finished.
template <bool COUNT>
static __device__ bool track_own(const SceneView& S, const MaskView& M, SegState& st, const LaneMem& lm, Work& wk) {
    Prop pr;
    begin_prop(pr, st);
    if (st.live) lane_propose<COUNT>(S, M, st, pr, lm, wk);
    return close_window<COUNT>(S, M, st, pr, lm, wk);
}

// Radiance of one camera ray over spp samples, with a constant environment.
// Single scattering: the camera segment is free-flight sampled (and its
// transmittance estimated on the same points, or exactly); a real collision
// scatters isotropically and estimates the transmittance of the way out.
// Multiple scattering: free flights from segment to segment with
// Henyey-Greenstein scattering until escape or max_scatter scatterings.
// Every segment traces the fixed mask or draws its own stochastic cell
// weights; with shadow_cells the shadow segment traces those cells of the
// fixed mask (Zero-NEE).  The camera segment draws from the sample's stream
// (seed, ray, sample, 0), the rest of its path from (seed, ray, sample, 2).
template <bool EXACT>
struct RenderLane {
    const float* r;
    float* wl;  // LDS cell-weight rows of this lane
    uint32_t key;
    int nsc, seg;
    int cs;  // the sample being traced
    bool shadow;
    float w, L;
    SampleSums acc;
    Rng g;
    SegState st;
    __device__ void begin(const float* ray, uint32_t k, float* cw_rows) {
        r = ray;
        wl = cw_rows;
        key = k;
        acc.zero();
    }
    __device__ CellW weights(const SceneView& S, const MaskView& M, const RenderArgs& A, const float* d) {
        return A.stochastic ? stochastic_weights(S, A.strat, M.cells, d[0], d[1], d[2], g, wl)
                            : fixed_weights(M.cells, wl);
    }
    // camera segment of sample s
    __device__ void start(const SceneView& S, const MaskView& M, const RenderArgs& A, int s) {
        cs = s;
        g.init(A.seed, key, (uint32_t)s, 0u);
        CellW cw = weights(S, M, A, r + 3);
        begin_segment(S, st, r, r + 3, r[6], r[7], cw, MODE_RATIO | MODE_DELTA, M.lod2, g);
        if (EXACT) draw_flight(st, g);
    }
    // after the camera segment: its transmittance estimate (summed, or
    // stored for the reduction when the ray's samples are split)
    __device__ void camera_done(const RenderArgs& A) {
        if (!A.part)
            acc.add_T(st.T);
        else if (A.keep_T)
            A.part[((size_t)A.spp + cs) * A.n + key] = st.T;
    }
    // the rest of sample s from its camera outcome (collision distance tc,
    // weight factor wf); true when the sample is already over
    __device__ bool begin_path(const SceneView& S, const MaskView& M, const RenderArgs& A, int s, float tc,
                               float wf) {
        cs = s;
        g.init(A.seed, key, (uint32_t)s, 2u);
        w = 1.0f;
        L = 0.0f;
        nsc = seg = 0;
        shadow = false;
        st.sg.ox = r[0];
        st.sg.oy = r[1];
        st.sg.oz = r[2];
        st.sg.vx = r[3];
        st.sg.vy = r[4];
        st.sg.vz = r[5];
        st.tc = tc;
        st.wf = wf;
        return segment_done(S, M, A);
    }
    __device__ bool end_sample(const RenderArgs& A) {
        if (A.part)
            A.part[(size_t)cs * A.n + key] = L;
        else
            acc.add_L(L);
        return true;
    }
    // Single scattering with a closed-form shadow transmittance in an image
    // launch: the rest of sample s from its camera outcome, with the
    // shadow direction drawn from the stream of the ray's 8x8 pixel tile
    // (seed, tile, sample, 3), shared by the tile's rays.  Each ray's
    // direction is still uniform on the sphere and independent of its
    // camera segment, so its estimate is unbiased; the tile's shadow rays
    // are parallel and trace as one packet.  Returns true when a shadow
    // segment was set up (false: the sample is over).
    __device__ bool begin_shadow(const SceneView& S, const MaskView& M, const RenderArgs& A, int s, float tc,
                                 float wf, uint32_t tile) {
        cs = s;
        g.init(A.seed, key, (uint32_t)s, 2u);
        L = 0.0f;
        nsc = seg = 0;
        w = wf;
        if (!(tc < INFINITY)) {
            L += w * A.env;
            shadow = false;
            end_sample(A);
            return false;
        }
        float x[3] = {r[0] + tc * r[3], r[1] + tc * r[4], r[2] + tc * r[5]};
        Rng gt;
        gt.init(A.seed, tile, (uint32_t)s, 3u);
        float d[3];
        sample_sphere(gt, d);
        shadow = true;
        seg = 1;
        CellW cw = A.shadow_cells ? fixed_weights(A.shadow_cells & M.cells, wl) : weights(S, M, A, d);
        begin_segment(S, st, x, d, 0.0f, INFINITY, cw, MODE_RATIO, 0.0f, g);
        return true;
    }
    // the current segment is finished: scatter (and set up the next
    // segment) or close the sample; true when the sample is over
    __device__ bool segment_done(const SceneView& S, const MaskView& M, const RenderArgs& A) {
        if (shadow) {
            L += w * A.albedo * st.T * A.env;
            return end_sample(A);
        }
        w *= st.wf;
        if (!(st.tc < INFINITY)) {
            L += w * A.env;
            return end_sample(A);
        }
        float x[3] = {st.sg.ox + st.tc * st.sg.vx, st.sg.oy + st.tc * st.sg.vy, st.sg.oz + st.tc * st.sg.vz};
        float d[3];
        int mode;
        if (!A.multiple) {
            sample_sphere(g, d);
            shadow = true;
            mode = MODE_RATIO;
        } else {
            if (nsc >= A.max_scatter) return end_sample(A);
            ++nsc;
            w *= A.albedo;
            float vn = rsqrtf(st.sg.vx * st.sg.vx + st.sg.vy * st.sg.vy + st.sg.vz * st.sg.vz);
            float wi[3] = {st.sg.vx * vn, st.sg.vy * vn, st.sg.vz * vn};
            sample_hg(g, A.hg, wi, d);
            mode = MODE_DELTA;
        }
        ++seg;
        CellW cw = (shadow && A.shadow_cells) ? fixed_weights(A.shadow_cells & M.cells, wl) : weights(S, M, A, d);
        begin_segment(S, st, x, d, 0.0f, INFINITY, cw, mode, 0.0f, g);
        if (EXACT && mode == MODE_DELTA) draw_flight(st, g);
        return false;
    }
    __device__ void result(const RenderArgs& A, float* out4) const { acc.result(A.spp, out4); }
};

// One wave renders samples [sb, se) of 64 rays (idx < 0: no ray on this
// lane), SG samples at a time: the camera segments of each sample go through the packet passes
// together (their outcomes kept in the workspace), then every lane follows
// the paths of its SG samples back to back with per-lane passes, so a lane
// with short paths does not wait on the longest path of each sample.
// FF: 0 delta tracking with ratio-tracked transmittances, 1 delta tracking
// with closed-form shadow transmittances, 2 CDF inversion with closed-form
// transmittances.
template <bool COUNT, int FF>
static __device__ void render_rays(const SceneView& S, const MaskView& M, const RenderArgs& A,
                                   const float* __restrict__ rays, int idx, int sb, int se, const LaneMem& lm,
                                   int* pstk, Work& wk, float* out4) {
    const bool valid = idx >= 0;
    constexpr bool EXACT = FF == 2;
    RenderLane<EXACT> rl;
    if (valid) rl.begin(rays + (size_t)idx * 8, (uint32_t)idx, lm.cw);
    for (int s0 = sb; s0 < se; s0 += SG) {
        const int gn = min(SG, se - s0);
        for (int k = 0; k < gn; ++k) {
            if (valid) rl.start(S, M, A, s0 + k);
            if (EXACT)
                exact_segment<COUNT, true>(S, M, rl.st, valid, lm, pstk, wk);
            else
                track_camera<COUNT, FF == 1>(S, M, rl.st, valid, lm, pstk, wk);
            if (valid) {
                rl.camera_done(A);
                lm.ctc(k) = rl.st.tc;
                lm.cwf(k) = rl.st.wf;
            }
        }
        if (FF == 1 && !A.multiple && A.tile_w > 0) {
            // shadow segments of the group's samples as packets
            const uint32_t tile = valid ? (uint32_t)((idx / A.tile_w >> 3) * (A.tile_w >> 3) + (idx % A.tile_w >> 3)) : 0u;
            for (int k = 0; k < gn; ++k) {
                const bool sh = valid && rl.begin_shadow(S, M, A, s0 + k, lm.ctc(k), lm.cwf(k), tile);
                exact_T_packet<COUNT>(S, M, rl.st, sh, lm, pstk, wk);
                if (sh) rl.segment_done(S, M, A);
            }
            continue;
        }
        int k = 0;
        // the next sample of the group whose path goes on past the camera
        auto next = [&]() {
            while (k < gn) {
                bool over = rl.begin_path(S, M, A, s0 + k, lm.ctc(k), lm.cwf(k));
                ++k;
                if (!over) return true;
            }
            return false;
        };
        bool more = valid && next();
        while (__any(more)) {
            if (more) {
                bool fin;
                if (rl.shadow && FF >= 1) {
                    // transmittance only: one closed-form pass, no bins
                    exact_T_own<COUNT>(S, M, rl.st, lm, wk);
                    fin = true;
                } else if (EXACT) {
                    exact_segment<COUNT, false>(S, M, rl.st, true, lm, pstk, wk);
                    fin = true;
                } else {
                    fin = track_own<COUNT>(S, M, rl.st, lm, wk);
                }
                if (fin && rl.segment_done(S, M, A)) more = next();
            }
        }
    }
    if (valid) rl.result(A, out4);
}

// Ratio-tracking transmittance of 64 rays over [tmin, tmax], spp samples.
template <bool COUNT>
static __device__ void ratio_rays(const SceneView& S, const MaskView& M, const float* __restrict__ rays, int idx,
                                  int spp, uint64_t seed, const LaneMem& lm, int* pstk, Work& wk, float* out2) {
    const bool valid = idx >= 0;
    const float* r = rays + (size_t)(valid ? idx : 0) * 8;
    float s1 = 0.0f, s2 = 0.0f;
    SegState st;
    for (int s = 0; s < spp; ++s) {
        if (valid) {
            Rng g;
            g.init(seed, (uint32_t)idx, (uint32_t)s, 1u);
            begin_segment(S, st, r, r + 3, r[6], r[7], fixed_weights(M.cells, lm.cw), MODE_RATIO, M.lod2, g);
        }
        track_camera<COUNT, false>(S, M, st, valid, lm, pstk, wk);
        s1 += st.T;
        s2 += st.T * st.T;
    }
    out2[0] = s1 / spp;
    out2[1] = spp > 1 ? fmaxf(0.0f, (s2 - s1 * s1 / spp) / (spp - 1)) : 0.0f;
}

// Work distribution: waves take chunks of 64 rays (one 8x8 tile of an image,
// or 64 consecutive rays) from a launch-wide counter.
static __device__ __forceinline__ int next_chunk(unsigned* counter) {
    unsigned c = 0;
    if (lane_id() == 0) c = atomicAdd(counter, 1u);
    return uniform_int((int)__shfl(c, 0));
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TR_THREADS) void k_density(SceneView S, MaskView M, const float* __restrict__ pts, int n,
                                                        float* __restrict__ kappa, float* __restrict__ kbar) {
    __shared__ int stk[TR_STACK * TR_THREADS];
    int i = blockIdx.x * TR_THREADS + threadIdx.x;
    if (i >= n) return;
    float x = pts[3 * (size_t)i], y = pts[3 * (size_t)i + 1], z = pts[3 * (size_t)i + 2];
    Work wk{};
    kappa[i] = point_density<false>(S, M, x, y, z, stk + threadIdx.x, wk);
    if (kbar) {
        float kb = 0.0f;
        if (x >= S.glo[0] && x <= S.ghi[0] && y >= S.glo[1] && y <= S.ghi[1] && z >= S.glo[2] && z <= S.ghi[2]) {
            int ix = min(S.G - 1, max(0, (int)floorf((x - S.glo[0]) * S.ginv[0])));
            int iy = min(S.G - 1, max(0, (int)floorf((y - S.glo[1]) * S.ginv[1])));
            int iz = min(S.G - 1, max(0, (int)floorf((z - S.glo[2]) * S.ginv[2])));
            float mw[GF_NCELLS];
            for (int c = 0; c < GF_NCELLS; ++c) mw[c] = ((M.cells >> c) & 1u) ? 1.0f : 0.0f;
            kb = voxel_majorant(S, (iz * S.G + iy) * S.G + ix, mw);
        }
        kbar[i] = kb;
    }
}

// The first 256 B of the workspace hold the launch's chunk counter (zeroed by
// k_zero before the launch); the lanes' slices follow.
#define WS_HEAD GF_TRACK_HEAD_FLOATS

__global__ void k_zero(unsigned* p) { *p = 0u; }

__global__ __launch_bounds__(TR_THREADS) void k_ratio(SceneView S, MaskView M, const float* __restrict__ rays, int n,
                                                      int tile_w, int nchunks, int spp, uint64_t seed,
                                                      float* __restrict__ ws, float* __restrict__ Tm,
                                                      float* __restrict__ Tv) {
    LANE_MEM(ws + WS_HEAD)
    __shared__ int pstk[TR_STACK];
    Work wk{};
    for (int c = next_chunk((unsigned*)ws); c < nchunks; c = next_chunk((unsigned*)ws)) {
        int idx = ray_of_tr(tile_order(c, nchunks, tile_w) * TR_THREADS + (int)threadIdx.x, n, tile_w);
        float o[2];
        ratio_rays<false>(S, M, rays, idx, spp, seed, lm, pstk, wk, o);
        if (idx >= 0) {
            Tm[idx] = o[0];
            if (Tv) Tv[idx] = o[1];
        }
    }
}

// Work units: chunk c of 64 rays (an 8x8 tile in an image launch) times
// A.groups sample groups of A.su samples, the groups of a chunk next to each
// other in the unit order.  With one group a unit writes its rays' results;
// with more, every sample's L and T go to A.part and k_render_reduce sums
// them.  Splitting a chunk's samples over several waves keeps the chip busy
// to the end of a launch whose few densest tiles cost far more than the rest.
// The CDF-inversion instance asks for at least two waves per SIMD: without
// the bound it takes more than 256 registers and runs one wave per SIMD.
// The other instances fit two waves without it, and the bound costs them
// 7-10% (the register allocator then trades registers for reloads).
template <bool COUNT, int FF>
__global__ __launch_bounds__(TR_THREADS) __attribute__((amdgpu_waves_per_eu(FF == 2 ? 2 : 1))) void k_render(SceneView S, MaskView M, const float* __restrict__ rays, int n,
                                                       int tile_w, int nchunks, RenderArgs A, float* __restrict__ ws,
                                                       float* __restrict__ Lm, float* __restrict__ Lv,
                                                       float* __restrict__ Tm, float* __restrict__ Tv,
                                                       unsigned long long* __restrict__ counters) {
    LANE_MEM(ws + WS_HEAD)
    __shared__ int pstk[TR_STACK];
    Work wk{};
    const int nunits = nchunks * A.groups;
    for (int u = next_chunk((unsigned*)ws); u < nunits; u = next_chunk((unsigned*)ws)) {
        const int c = u / A.groups, sb = (u - c * A.groups) * A.su, se = min(A.spp, sb + A.su);
        int idx = ray_of_tr(tile_order(c, nchunks, tile_w) * TR_THREADS + (int)threadIdx.x, n, tile_w);
        float o[4];
        render_rays<COUNT, FF>(S, M, A, rays, idx, sb, se, lm, pstk, wk, o);
        if (!COUNT && !A.part && idx >= 0) {
            Lm[idx] = o[0];
            if (Lv) Lv[idx] = o[1];
            if (Tm) Tm[idx] = o[2];
            if (Tv) Tv[idx] = o[3];
        }
    }
    if (COUNT) {
        atomicAdd(counters + 0, wk.tent);
        atomicAdd(counters + 1, wk.nodes);
        atomicAdd(counters + 2, wk.prims);
        atomicAdd(counters + 3, wk.windows);
        atomicAdd(counters + 4, wk.used);
        atomicAdd(counters + 5, wk.pq_nodes);
        atomicAdd(counters + 6, wk.cover);
    }
}

// Per-ray mean and variance of split samples: part holds spp x n values of
// L, then spp x n of T (sample-major), summed in sample order as a lane
// sums them.
__global__ __launch_bounds__(256) void k_render_reduce(const float* __restrict__ part, int n, int spp,
                                                       float* __restrict__ Lm, float* __restrict__ Lv,
                                                       float* __restrict__ Tm, float* __restrict__ Tv) {
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= n) return;
    SampleSums a;
    a.zero();
    for (int s = 0; s < spp; ++s) a.add_L(part[(size_t)s * n + i]);
    for (int s = 0; s < spp; ++s) a.add_T(part[((size_t)spp + s) * n + i]);
    float o[4];
    a.result(spp, o);
    Lm[i] = o[0];
    if (Lv) Lv[i] = o[1];
    if (Tm) Tm[i] = o[2];
    if (Tv) Tv[i] = o[3];
}

// Serving: one launch renders tiles of many requests (each tile a contiguous
// range of one request's rays, cut into chunks of 64).  A work unit is one
// sample of one chunk: the units of tile t start at tiles[t].unit0, chunk by
// chunk, the request's samples of a chunk next to each other.  Every sample's
// L goes to the request's per-sample buffer (spp x n floats) and
// k_serve_reduce sums a tile's samples once the launch is over.  A request's
// random streams are keyed by its own seed and pixel index and a lane's
// result does not depend on the other rays of its chunk, so its image does
// not depend on the batch.
struct ServeReq {
    SceneView S;
    MaskView M;
    RenderArgs A;
    const float* rays;
    float* out;
    int n;
};

struct ServeTile {
    int req, first, count, unit0;
};

// the tile holding unit u (tiles in unit order)
static __device__ __forceinline__ int serve_tile_of(const ServeTile* __restrict__ tiles, int ntiles, int u) {
    int lo = 0, hi = ntiles - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tiles[mid].unit0 <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(TR_THREADS) void k_render_tiles(const ServeReq* __restrict__ reqs,
                                                             const ServeTile* __restrict__ tiles, int ntiles,
                                                             int nunits, float* __restrict__ ws) {
    LANE_MEM(ws + WS_HEAD)
    __shared__ int pstk[TR_STACK];
    Work wk{};
    for (int u = next_chunk((unsigned*)ws); u < nunits; u = next_chunk((unsigned*)ws)) {
        const ServeTile tl = tiles[serve_tile_of(tiles, ntiles, u)];
        const ServeReq& R = reqs[tl.req];
        const int v = u - tl.unit0, chunk = v / R.A.spp, smp = v - chunk * R.A.spp;
        const int local = chunk * TR_THREADS + (int)threadIdx.x;
        const int idx = local < tl.count ? tl.first + local : -1;
        float o[4];
        render_rays<false, 0>(R.S, R.M, R.A, R.rays, idx, smp, smp + 1, lm, pstk, wk, o);
    }
}

// mean radiance of every ray of a launch's tiles from the stored samples
// (one thread per ray slot of tile_rays per tile)
__global__ __launch_bounds__(256) void k_serve_reduce(const ServeReq* __restrict__ reqs,
                                                      const ServeTile* __restrict__ tiles, int tile_rays,
                                                      int64_t nslots) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nslots) return;
    const ServeTile tl = tiles[i / tile_rays];
    const int local = (int)(i % tile_rays);
    if (local >= tl.count) return;
    const ServeReq& R = reqs[tl.req];
    const int idx = tl.first + local, spp = R.A.spp;
    SampleSums a;
    a.zero();
    for (int s = 0; s < spp; ++s) a.add_L(R.A.part[(size_t)s * R.n + idx]);
    float o[4];
    a.result(spp, o);
    R.out[idx] = o[0];
}

// ---------------------------------------------------------------------------
// workspace: WS_ROWS x TR_THREADS floats per resident wave
// ---------------------------------------------------------------------------
static unsigned res_blocks(int64_t nblocks) { return (unsigned)std::min<int64_t>(nblocks, TR_RES_BLOCKS); }

size_t gf_track_workspace_bytes(int64_t nblocks) {
    return ((size_t)WS_HEAD + (size_t)res_blocks(nblocks) * WS_ROWS * TR_THREADS) * sizeof(float);
}

static unsigned tr_blocks(int64_t n, int tile_w) {
    return (unsigned)((tr_threads(n, tile_w) + TR_THREADS - 1) / TR_THREADS);
}

static RenderArgs render_args(const gf_render_desc* d) {
    RenderArgs A;
    A.spp = d->spp;
    A.multiple = d->multiple;
    A.max_scatter = d->max_scatter;
    A.stochastic = d->stochastic;
    A.exact = d->free_flight;
    A.albedo = d->albedo;
    A.hg = d->hg_g;
    A.env = d->env;
    A.strat.level = d->level_strategy;
    A.strat.bin = d->bin_strategy;
    A.strat.beta = d->beta;
    A.strat.delta = d->delta;
    A.shadow_cells = (uint32_t)(d->shadow_cells & 0xFFFu);
    A.tile_w = 0;
    A.su = d->spp;
    A.groups = 1;
    A.n = 0;
    A.part = nullptr;
    A.keep_T = 1;
    A.seed = d->seed;
    return A;
}

gf_status gf_serve_fill_req(const gf_request* q, const float* rays, float* part, void* out_desc) {
    ServeReq* d = (ServeReq*)out_desc;
    d->S = gf_scene_view(q->scene);
    d->M = gf_mask_view(q->render.mask);
    d->A = render_args(&q->render);
    d->A.tile_w = q->camera.width % 8 == 0 ? q->camera.width : 0;  // as gf_render: the same image
    d->rays = rays;
    d->out = q->out;
    d->n = q->camera.width * q->camera.height;
    d->A.n = d->n;
    d->A.part = part;  // spp x n per-sample radiance
    d->A.keep_T = 0;
    return GF_OK;
}

size_t gf_serve_req_size() { return sizeof(ServeReq); }
size_t gf_serve_tile_size() { return sizeof(ServeTile); }
int gf_serve_tile_threads() { return TR_THREADS; }

size_t gf_serve_workspace_bytes(int max_tiles, int tile_rays) {
    int64_t bpt = (tile_rays + TR_THREADS - 1) / TR_THREADS;
    return gf_track_workspace_bytes((int64_t)max_tiles * bpt);
}

// A batch of ntiles tiles (nunits work units) in the workspace ws of a
// server created with max_tiles, then the per-ray means.
gf_status gf_serve_launch(const void* dreqs, const void* dtiles, int ntiles, int nunits, int tile_rays,
                          int max_tiles, float* ws, hipStream_t sm) {
    const int64_t bpt = (tile_rays + TR_THREADS - 1) / TR_THREADS;
    const unsigned g = std::min(res_blocks(nunits), res_blocks((int64_t)max_tiles * bpt));
    k_zero<<<1, 1, 0, sm>>>((unsigned*)ws);
    k_render_tiles<<<g, TR_THREADS, 0, sm>>>((const ServeReq*)dreqs, (const ServeTile*)dtiles, ntiles, nunits, ws);
    const int64_t slots = (int64_t)ntiles * tile_rays;
    k_serve_reduce<<<(unsigned)((slots + 255) / 256), 256, 0, sm>>>((const ServeReq*)dreqs, (const ServeTile*)dtiles,
                                                                    tile_rays, slots);
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
gf_status gf_check_track_depth(const gf_scene_s* s, const char* who) {
    if (s->depth > TR_STACK) return gf_fail(GF_EINVAL, "%s: LBVH depth %d exceeds the point-query stack", who, s->depth);
    return GF_OK;
}

// Stream-ordered workspace of one launch (freed on the same stream after it).
struct Workspace {
    float* p = nullptr;
    float* part = nullptr;  // per-sample buffer after the tracking slices (part_floats > 0)
    hipStream_t sm = nullptr;
    gf_status alloc(int64_t nblocks, size_t part_floats, hipStream_t s, const char* who) {
        sm = s;
        const size_t track = (gf_track_workspace_bytes(nblocks) + 255) & ~(size_t)255;
        size_t bytes = track + part_floats * sizeof(float);
        hipError_t e = hipMallocAsync((void**)&p, bytes, sm);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return gf_fail(GF_ENOMEM, "%s: workspace of %zu bytes: %s", who, bytes, hipGetErrorString(e));
        }
        if (part_floats) part = (float*)((char*)p + track);
        return GF_OK;
    }
    ~Workspace() {
        if (p) (void)hipFreeAsync(p, sm);
    }
};

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
    if (kbar && s->G == 0) return gf_fail(GF_EINVAL, "gf_density: kbar needs a scene built with a majorant grid");
    gf_status st = gf_check_track_depth(s, "gf_density");
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
    if (st == GF_OK) st = gf_check_track_depth(s, "gf_transmittance_ratio");
    if (st == GF_OK && n > 0) st = gf_validate_rays(rays, n, (hipStream_t)stream, "gf_transmittance_ratio");
    if (st != GF_OK || n == 0) return st;
    unsigned nb = tr_blocks(n, image_width);
    Workspace ws;
    st = ws.alloc(nb, 0, (hipStream_t)stream, "gf_transmittance_ratio");
    if (st != GF_OK) return st;
    k_zero<<<1, 1, 0, (hipStream_t)stream>>>((unsigned*)ws.p);
    k_ratio<<<res_blocks(nb), TR_THREADS, 0, (hipStream_t)stream>>>(gf_scene_view(s), gf_mask_view(mask), rays, (int)n,
                                                                    image_width, (int)nb, spp, seed, ws.p, T_mean,
                                                                    T_var);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

// Samples per work unit: one.  A chunk's samples then run on as many waves
// as the chip has free, which keeps it busy to the end of a launch whose
// few densest tiles cost far more than the rest; measured on blob100k it
// beats units of 8 samples (whose lanes chain the secondary paths of their
// samples) on every render: camera segments 2.9x, CDF inversion 3.0x,
// ratio-tracked shadows 1.4x, multiple scattering 1.2x.
static int render_su(const gf_render_desc*, int) { return 1; }

// Largest per-sample buffer a render uses (floats); beyond it the samples of
// a chunk stay in one unit.
#define PART_MAX_FLOATS ((size_t)1 << 28)

// Floats of per-sample storage the render of n rays splits its samples
// into (0: one unit per chunk, no storage).
size_t gf_render_part_floats(const gf_render_desc* d, int64_t n, int tile_w) {
    const int su = render_su(d, tile_w);
    const int64_t groups = ((int64_t)d->spp + su - 1) / su;
    if (groups <= 1 || (int64_t)tr_blocks(n, tile_w) * groups > (int64_t)INT32_MAX / 2) return 0;
    const size_t f = (size_t)2 * (size_t)d->spp * (size_t)n;
    return f <= PART_MAX_FLOATS ? f : 0;
}

// Tracking slices (resident waves) of a render of n rays: one per work
// unit, at most TR_RES_BLOCKS.  Workspaces hold this many, and a launch
// never uses more waves than its workspace holds.
int64_t gf_render_waves(const gf_render_desc* d, int64_t n, int tile_w) {
    const int64_t nb = tr_blocks(n, tile_w);
    const int su = render_su(d, tile_w);
    const int64_t groups = gf_render_part_floats(d, n, tile_w) ? ((int64_t)d->spp + su - 1) / su : 1;
    return res_blocks(nb * groups);
}

// Launch of the render kernel over n rays with the tracking workspace ws
// (ws_waves slices after its head) and the per-sample buffer part of
// part_cap floats (NULL / too small: one unit per chunk; the results have
// the same bits either way).
static gf_status render_launch(gf_scene s, const float* rays, int64_t n, int image_width, const gf_render_desc* d,
                               float* ws, int64_t ws_waves, float* part, size_t part_cap, float* L_mean,
                               float* L_var, float* T_mean, float* T_var, hipStream_t sm,
                               unsigned long long* counters) {
    RenderArgs A = render_args(d);
    A.tile_w = image_width;
    const int ff = A.exact ? 2 : (d->transmittance ? 1 : 0);
    if (ff) {
        gf_status st = gf_ensure_weideman_track();
        if (st != GF_OK) return st;
    }
    const size_t pf = gf_render_part_floats(d, n, image_width);
    const bool split = pf > 0 && (counters || (part && part_cap >= pf));
    A.su = split ? render_su(d, image_width) : d->spp;
    A.groups = (d->spp + A.su - 1) / A.su;
    A.n = (int)n;
    A.part = split && !counters ? part : nullptr;
    unsigned nb = tr_blocks(n, image_width);
    int total = (int)nb;  // chunks of TR_THREADS rays
    k_zero<<<1, 1, 0, sm>>>((unsigned*)ws);
    const SceneView S = gf_scene_view(s);
    const MaskView M = gf_mask_view(d->mask);
    const unsigned g = (unsigned)std::min<int64_t>(res_blocks((int64_t)nb * A.groups), ws_waves);
    auto launch = [&](auto kernel, float* a, float* b, float* c, float* e, unsigned long long* cnt) {
        kernel<<<g, TR_THREADS, 0, sm>>>(S, M, rays, (int)n, image_width, total, A, ws, a, b, c, e, cnt);
    };
    if (counters) {
        if (ff == 0) launch(k_render<true, 0>, nullptr, nullptr, nullptr, nullptr, counters);
        if (ff == 1) launch(k_render<true, 1>, nullptr, nullptr, nullptr, nullptr, counters);
        if (ff == 2) launch(k_render<true, 2>, nullptr, nullptr, nullptr, nullptr, counters);
    } else {
        if (ff == 0) launch(k_render<false, 0>, L_mean, L_var, T_mean, T_var, nullptr);
        if (ff == 1) launch(k_render<false, 1>, L_mean, L_var, T_mean, T_var, nullptr);
        if (ff == 2) launch(k_render<false, 2>, L_mean, L_var, T_mean, T_var, nullptr);
        if (A.part)
            k_render_reduce<<<(unsigned)((n + 255) / 256), 256, 0, sm>>>(A.part, (int)n, d->spp, L_mean, L_var,
                                                                          T_mean, T_var);
    }
    GF_HIP(hipGetLastError());
    return GF_OK;
}

gf_status gf_render_launch(gf_scene s, const float* rays, int64_t n, int image_width, const gf_render_desc* d,
                           float* L_mean, float* L_var, float* T_mean, float* T_var, hipStream_t sm,
                           unsigned long long* counters) {
    const size_t pf = counters ? 0 : gf_render_part_floats(d, n, image_width);
    const int64_t waves = gf_render_waves(d, n, image_width);
    Workspace ws;
    gf_status st = ws.alloc(waves, pf, sm, "gf_render_rays");
    if (st != GF_OK) return st;
    return render_launch(s, rays, n, image_width, d, ws.p, waves, ws.part, pf, L_mean, L_var, T_mean, T_var, sm,
                         counters);
}

gf_status gf_check_render_desc(const gf_render_desc* d, const char* who) {
    if (!d) return gf_fail(GF_EINVAL, "%s: NULL desc", who);
    if (d->spp < 1 || d->max_scatter < 0) return gf_fail(GF_EINVAL, "%s: spp >= 1 and max_scatter >= 0 required", who);
    if (!isfinite(d->albedo) || !isfinite(d->hg_g) || !(fabsf(d->hg_g) < 1.0f) || !isfinite(d->env))
        return gf_fail(GF_EINVAL, "%s: albedo / hg_g / env invalid", who);
    if (d->stochastic) {
        if (d->level_strategy < GF_LEVEL_ALL || d->level_strategy > GF_LEVEL_POWER_CV_ACCUM)
            return gf_fail(GF_EINVAL, "%s: unknown level strategy %d", who, d->level_strategy);
        if (d->bin_strategy < GF_BIN_ALL || d->bin_strategy > GF_BIN_MIXTURE)
            return gf_fail(GF_EINVAL, "%s: unknown bin strategy %d", who, d->bin_strategy);
        if (!(d->beta >= 0.0f && d->beta < 1.0f)) return gf_fail(GF_EINVAL, "%s: beta must lie in [0, 1)", who);
        if (!(d->delta >= 0.0f && d->delta <= 1.0f)) return gf_fail(GF_EINVAL, "%s: delta must lie in [0, 1]", who);
    }
    if (d->free_flight != 0 && d->free_flight != 1) return gf_fail(GF_EINVAL, "%s: free_flight must be 0 or 1", who);
    if (d->transmittance != 0 && d->transmittance != 1)
        return gf_fail(GF_EINVAL, "%s: transmittance must be 0 or 1", who);
    if (!(d->mask.lod_k >= 0.0f) || !isfinite(d->mask.lod_k)) return gf_fail(GF_EINVAL, "%s: lod_k must be >= 0", who);
    return GF_OK;
}

// Argument checks shared by the ray-list render calls.
static gf_status check_render_rays(gf_scene s, const float* rays, int64_t n, int image_width, const gf_render_desc* d,
                                   hipStream_t sm, const char* who) {
    gf_status st = gf_check_render_desc(d, who);
    if (st == GF_OK) st = check_rays_tr(n, image_width, who);
    if (st == GF_OK) st = gf_check_track_depth(s, who);
    if (st == GF_OK && n > 0) st = gf_validate_rays(rays, n, sm, who);
    return st;
}

extern "C" gf_status gf_render_rays(gf_scene s, const float* rays, int64_t n, int image_width, const gf_render_desc* d,
                                    float* L_mean, float* L_var, float* T_mean, float* T_var, void* stream) {
    if (!s || (n && (!rays || !L_mean))) return gf_fail(GF_EINVAL, "gf_render_rays: NULL argument");
    hipStream_t sm = (hipStream_t)stream;
    gf_status st = check_render_rays(s, rays, n, image_width, d, sm, "gf_render_rays");
    if (st != GF_OK || n == 0) return st;
    return gf_render_launch(s, rays, n, image_width, d, L_mean, L_var, T_mean, T_var, sm, nullptr);
}

extern "C" gf_status gf_render_counts(gf_scene s, const float* rays, int64_t n, int image_width,
                                      const gf_render_desc* d, uint64_t* counts, void* stream) {
    if (!s || !counts || (n && !rays)) return gf_fail(GF_EINVAL, "gf_render_counts: NULL argument");
    hipStream_t sm = (hipStream_t)stream;
    gf_status st = check_render_rays(s, rays, n, image_width, d, sm, "gf_render_counts");
    if (st != GF_OK) return st;
    st = gf_zero_words(counts, 2 * GF_RENDER_COUNTS, sm);
    if (st != GF_OK || n == 0) return st;
    return gf_render_launch(s, rays, n, image_width, d, nullptr, nullptr, nullptr, nullptr, sm,
                            (unsigned long long*)counts);
}

// Camera render: the caller's workspace holds the camera rays (n x 32 B,
// 256-byte aligned), the tracking workspace, then the per-sample buffer.
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static gf_status camera_render_bytes(const gf_camera* cam, const gf_render_desc* d, size_t* rays_bytes,
                                     size_t* track_bytes, size_t* part_floats, size_t* total) {
    const int64_t n = (int64_t)cam->width * cam->height;
    const int tile_w = cam->width % 8 == 0 ? cam->width : 0;
    *rays_bytes = align256((size_t)n * 8 * sizeof(float));
    *track_bytes = align256(gf_track_workspace_bytes(gf_render_waves(d, n, tile_w)));
    *part_floats = gf_render_part_floats(d, n, tile_w);
    *total = *rays_bytes + *track_bytes + align256(*part_floats * sizeof(float));
    return GF_OK;
}

extern "C" gf_status gf_render_workspace_size(gf_scene s, const gf_camera* cam, const gf_render_desc* d,
                                              size_t* bytes) {
    gf_status st = gf_check_camera(cam, "gf_render_workspace_size");
    if (st == GF_OK) st = gf_check_render_desc(d, "gf_render_workspace_size");
    if (st != GF_OK) return st;
    if (!s || !bytes) return gf_fail(GF_EINVAL, "gf_render_workspace_size: NULL argument");
    size_t rb, tb, pf;
    return camera_render_bytes(cam, d, &rb, &tb, &pf, bytes);
}

extern "C" gf_status gf_render(gf_scene s, const gf_camera* cam, const gf_render_desc* d, void* workspace,
                               size_t ws_bytes, float* radiance, float* primary_T, void* stream) {
    gf_status st = gf_check_camera(cam, "gf_render");
    if (st == GF_OK) st = gf_check_render_desc(d, "gf_render");
    if (st != GF_OK) return st;
    if (!s || !workspace || !radiance) return gf_fail(GF_EINVAL, "gf_render: NULL argument");
    st = gf_check_track_depth(s, "gf_render");
    if (st != GF_OK) return st;
    if (((uintptr_t)workspace & 255u) != 0) return gf_fail(GF_EINVAL, "gf_render: workspace must be 256-byte aligned");
    size_t rb, tb, pf, need;
    camera_render_bytes(cam, d, &rb, &tb, &pf, &need);
    if (ws_bytes < need)
        return gf_fail(GF_EINVAL, "gf_render: workspace of %zu bytes, %zu needed", ws_bytes, need);
    hipStream_t sm = (hipStream_t)stream;
    const int64_t n = (int64_t)cam->width * cam->height;
    const int tile_w = cam->width % 8 == 0 ? cam->width : 0;
    float* rays = (float*)workspace;
    st = gf_camera_launch(cam, rays, sm);
    if (st != GF_OK) return st;
    return render_launch(s, rays, n, tile_w, d, (float*)((char*)workspace + rb), gf_render_waves(d, n, tile_w),
                         (float*)((char*)workspace + rb + tb), pf, radiance, nullptr, primary_T, nullptr, sm, nullptr);
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

gf_status gf_render_launch_in(gf_scene s, const float* rays, int64_t n, int image_width, const gf_render_desc* d,
                              float* ws, int64_t ws_waves, float* part, size_t part_cap, float* radiance,
                              float* primary_T, hipStream_t sm) {
    return render_launch(s, rays, n, image_width, d, ws, ws_waves, part, part_cap, radiance, nullptr, primary_T,
                         nullptr, sm, nullptr);
}
