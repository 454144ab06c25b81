/*
 * gaborfields.h - C ABI of the MI355X (gfx950) Gabor-field rendering library.
 *
 * The library traces rays through a volumetric density that is a mixture of
 * anisotropic Gabor kernels (paper: "Gabor Fields: Orientation-Selective
 * Level-of-Detail for Volume Rendering"; Sec. 3 for the extinction field,
 * optical depth and transmittance, Sec. 4.2 for the kernel, Sec. 4.4 for the
 * closed-form line integral, Sec. 4.5 for frequency / orientation masking).
 *
 * Conventions shared by every call
 * --------------------------------
 * Primitive record: 15 float32 per primitive, array of structs, in the
 *   caller's order:  mu[3]  q[4] (w,x,y,z; rotation local->world)  s[3]
 *   f[3] (carrier frequency, cycles per unit)  phi (carrier phase, rad)  alpha.
 *   Kernel: g(x) = (2 pi)^-3/2 / (s0 s1 s2) * exp(-M/2) * cos(2 pi f.(x-mu) + phi)
 *   for M = (x-mu)^T Sigma^-1 (x-mu) < r^2, else 0;  Sigma = R S^2 R^T.
 *   Extinction kappa(x) = rho * sum_i alpha_i g_i(x)  (signed).
 * Ray record: 8 float32 per ray: o[3] v[3] tmin tmax, x(t) = o + t v; v need
 *   not be unit length (optical depth is in the units of t); tmax may be +inf.
 * Masks: the 12 cells are (frequency level l in 0..3) x (orientation bin k in
 *   0..2), cell = 3 l + k.  Level: |f|^2 <= fmax^2/64 -> 0, <= fmax^2/16 -> 1,
 *   <= fmax^2/4 -> 2, else 3 (fmax the largest |f| of the scene); bin: the axis
 *   of the largest |f_k| (ties to the lower axis).  A gf_mask keeps primitive i
 *   when bit cell(i) of `cells` is set AND (prim_bits == NULL or bit i of
 *   prim_bits is set).  This follows the per-level visibility masks V_l = 2^l
 *   and the ray-mask AND of Sec. 4.5 (implementation details).
 * Pointers: every array argument documented "device" is device memory of the
 *   current HIP device, owned by the caller; the library never frees it.
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Calls are
 *   stream-ordered and asynchronous unless documented otherwise.
 * Errors: every call returns a gf_status; on a non-OK status gf_last_error()
 *   returns a thread-local message.  Invalid arguments are rejected before any
 *   kernel is launched.  Nothing throws across this interface.
 */
#ifndef GABORFIELDS_H
#define GABORFIELDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GF_OK = 0,
    GF_EINVAL = -1,  /* invalid argument (shape, NaN/Inf, scale <= 0, |q| = 0, |v| = 0, tmin > tmax) */
    GF_ENOMEM = -2,  /* device allocation failed */
    GF_EDEVICE = -3, /* HIP runtime error */
    GF_ESTATE = -4,  /* object in the wrong state (e.g. destroyed server) */
    GF_EBUSY = -5    /* request does not fit the server's memory budget right now */
} gf_status;

typedef struct gf_scene_s* gf_scene;

typedef struct {
    float rho;          /* extinction scale multiplying every alpha (> 0) */
    float trunc_r;      /* Mahalanobis truncation radius r (Sec. 3: 3-sigma support); 0 -> 3 */
    int majorant_grid;  /* majorant grid resolution G (G^3 voxels); 0 -> 64 */
} gf_scene_desc;

typedef struct {
    uint64_t cells;            /* bit c keeps cell c (c = 3*level + bin); bits >= 12 ignored */
    const uint32_t* prim_bits; /* device, ceil(n/32) words, caller order; NULL = all */
} gf_mask;

typedef struct {
    int64_t n;
    float rho, trunc_r;
    double fmax;                 /* largest |f| */
    uint64_t nonempty_cells;     /* bit c set when cell c holds a primitive */
    int64_t cell_count[12];      /* primitives per cell */
    float cell_median_kw[12];    /* lower median of |k_W| = |S R^T omega| per cell (0 if empty) */
    int grid_res;
    float bounds_lo[3], bounds_hi[3]; /* box of all truncated ellipsoids */
    size_t device_bytes;         /* device memory held by the scene */
} gf_scene_info_t;

/* Builds a resident scene: validates the records, derives the per-primitive
 * constants, builds the Morton-ordered LBVH over the truncated ellipsoids and
 * the majorant grid.  params: device, n x 15 float32 (read only during the
 * call).  Synchronises `stream` once to report invalid input.  The scene
 * owns its device memory until gf_scene_destroy.
 * LBVH (bit-exact specification): scene bounds lo/hi = min/max of the float32
 * means; q_a = min(2^21-1, floor((mu_a - lo_a) * (2^21 / (hi_a - lo_a)))) in
 * binary64 (0 if hi_a == lo_a); key bits 3k+2, 3k+1, 3k = x_k, y_k, z_k;
 * stable sort by (key, index); Karras radix tree (delta = clz64 of key xor,
 * 64 + clz32 of index xor for equal keys); leaf box mu -/+ r sqrt(diag Sigma)
 * rounded outward to float32; internal boxes and cell masks are unions. */
gf_status gf_scene_create(const float* params, int64_t n, const gf_scene_desc* desc, void* stream,
                          gf_scene* out);
gf_status gf_scene_destroy(gf_scene scene);
gf_status gf_scene_info(gf_scene scene, gf_scene_info_t* info);

/* Copies the canonical LBVH into caller device buffers (any may be NULL):
 * keys[n] (sorted Morton keys), perm[n] (sorted leaf j -> caller index),
 * left/right[n-1] (child node ids; internal i -> i, leaf j -> n-1+j),
 * parent[2n-1] (-1 for the root), aabb[(2n-1) x 6] (lo xyz, hi xyz),
 * cellor[2n-1] (bit c set when the subtree holds cell c).  Stream-ordered. */
gf_status gf_scene_export_lbvh(gf_scene scene, uint64_t* keys, int32_t* perm, int32_t* left, int32_t* right,
                               int32_t* parent, float* aabb, uint64_t* cellor, void* stream);

/* cells[n] (device, caller order): the cell id 3*level + bin of every primitive. */
gf_status gf_scene_cells(gf_scene scene, int32_t* cells, void* stream);

/* Cell mask of an LOD level: 0 = all levels, 1 = levels 0..2 (1/2 band),
 * 2 = levels 0..1 (1/4 band), 3 = level 0 (1/8 band); all bins.  Host only. */
uint64_t gf_mask_lod_cells(int lod);

/* Orientation-cone mask (Sec. 4.5.2, threshold culling: the frequency
 * directions aligned with `axis` are removed): writes prim_bits (device,
 * ceil(n/32) words, caller order) with bit i set when
 * (f_i . a)^2 <= cos^2(half_angle) |f_i|^2, a = axis / |axis|. */
gf_status gf_mask_cone(gf_scene scene, const float axis[3], float half_angle, uint32_t* prim_bits,
                       void* stream);

/* Deterministic optical depth (Sec. 3, Eq. 2 summed over primitives, each by
 * the closed-form segment integral of Sec. 4.4) and transmittance T = exp(-tau)
 * (Sec. 3, Eq. 3; accumulate-then-exponentiate as in Sec. 4.5 implementation
 * details).  rays: device n x 8; tau: device n (required); T: device n or NULL.
 * image_width: 0 when the rays are an arbitrary list; W > 0 (a multiple of 8
 * dividing n) when they are a row-major image W pixels wide, which lets each
 * wave trace an 8x8 pixel tile.  Results do not depend on image_width. */
gf_status gf_optical_depth(gf_scene scene, const float* rays, int64_t n, int image_width, gf_mask mask,
                           float* tau, float* T, void* stream);

/* Traversal work of gf_optical_depth per ray (device int32 n each, either may
 * be NULL): boxes that met the ray (internal + leaf, root included) and
 * primitives whose truncated chord was non-empty.  Used to count algorithmic
 * bytes. */
gf_status gf_optical_depth_counts(gf_scene scene, const float* rays, int64_t n, int image_width, gf_mask mask,
                                  int32_t* nodes, int32_t* hits, void* stream);

/* Point density kappa (Sec. 3, Eq. 1) and the majorant-grid bound kbar at
 * points: pts device n x 3; kappa, kbar device n (kbar may be NULL). */
gf_status gf_density(gf_scene scene, const float* pts, int64_t n, gf_mask mask, float* kappa, float* kbar,
                     void* stream);

/* Ratio-tracking transmittance (Sec. 4.4 distance sampling; ratio tracking
 * of the voxel comparison): spp estimates per ray T_hat = prod_j (1 -
 * kappa(x_j)/kbar(x_j)) over tentative points of the per-ray envelope
 * majorant kbar(t) = sum_i rho |alpha_i| c_i exp(-M_i/2) of the masked
 * primitives the ray crosses (it bounds |kappa| term by term); outputs the
 * mean and the unbiased sample variance (T_var may be NULL).  Random
 * numbers: Philox4x32-10 streams keyed by (seed, ray, sample) and per chord
 * by (primitive, window, block); image_width as for gf_optical_depth.  The
 * scene's LBVH depth must not exceed 64 (checked).  Each ray's samples run
 * on one lane: for many samples of few rays, repeat the rays. */
gf_status gf_transmittance_ratio(gf_scene scene, const float* rays, int64_t n, int image_width, gf_mask mask,
                                 int spp, uint64_t seed, float* T_mean, float* T_var, void* stream);

typedef struct {
    int spp;            /* camera samples per ray */
    int multiple;       /* 0: single scattering, 1: multiple scattering */
    int max_scatter;    /* multiple: a collision after this many scatterings ends the path with 0 */
    float albedo;       /* single-scattering albedo */
    float hg_g;         /* Henyey-Greenstein asymmetry (0 = isotropic) */
    float env;          /* constant environment radiance */
    int stochastic;     /* 1: per-segment stochastic band / orientation mask (Sec. 4.5.1-4.5.2) */
    gf_mask mask;       /* fixed mask (stochastic == 0) */
    uint64_t seed;
} gf_render_desc;

/* Radiance per ray with signed-weight delta tracking (free flights) and
 * ratio tracking (shadow ray of single scattering; primary transmittance),
 * both against the per-ray envelope majorant of gf_transmittance_ratio.
 * Single: escape -> w env; real collision -> w albedo T_ratio(x, isotropic
 * direction) env.  Multiple: free flights with albedo and HG scattering until
 * escape.  Stochastic masks (Sec. 4.5.1-4.5.2, Appendix B tables): each
 * segment keeps level 0 (weight 1) and draws one level l in 1..3 uniformly
 * and one bin k with probability p_k = w_k / (2W) + 1/6 (an even mixture of
 * importance and uniform sampling), w_k = exp(-m_lk^2 a_k^2 / 2),
 * a_k = |v.e_k|, W = sum_k w_k, m_lk = cell median of |k_W|; the drawn cell
 * gets weight 3 / p_k (at most 18).
 * Outputs (device n, variances/T may be NULL): L mean / variance over spp,
 * primary-segment ratio-tracked transmittance mean / variance.
 * image_width as for gf_optical_depth.  Each ray's samples are traced by one
 * lane, so results do not depend on which rays are traced together. */
gf_status gf_render(gf_scene scene, const float* rays, int64_t n, int image_width, const gf_render_desc* desc,
                    float* L_mean, float* L_var, float* T_mean, float* T_var, void* stream);

/* Work of gf_render with the same arguments (same random streams):
 * counts[0] tentative collisions, [1] LBVH nodes visited by point queries,
 * [2] primitive records read at leaves, [3] majorant voxels walked.
 * counts: device, 4 x uint64, overwritten.  Used to count algorithmic bytes. */
gf_status gf_render_counts(gf_scene scene, const float* rays, int64_t n, int image_width, const gf_render_desc* desc,
                           uint64_t* counts, void* stream);

typedef struct {
    int kind;               /* 0 orthographic (rays along +z over [0,1]^2 at z0 = eye[2]), 1 pinhole */
    float eye[3], target[3], up[3];
    float fov_y_deg;
    int width, height;
} gf_camera;

/* Camera rays through pixel centres, row-major, top row first: device
 * width*height x 8 float32 (t in [0, +inf)). */
gf_status gf_camera_rays(const gf_camera* cam, float* rays, void* stream);

/* Adjoint of gf_optical_depth (and of T = exp(-tau)): accumulates
 * dparams[i*15 + k] = sum_r g_r dtau_r / dparam_{i,k} with
 * g_r = dL_dtau[r] - (dL_dT ? dL_dT[r] * T[r] : 0), by recomputing every
 * segment (no stored paths).  dparams: device n_prims x 15, caller order,
 * overwritten.  dL_dtau: device n; dL_dT and T: device n or both NULL.
 * Accumulation is float32 with atomics (not bitwise reproducible). */
gf_status gf_optical_depth_backward(gf_scene scene, const float* rays, int64_t n, int image_width, gf_mask mask,
                                    const float* dL_dtau, const float* dL_dT, const float* T, float* dparams,
                                    void* stream);

/* ------------------------------------------------------------------------- */
/* Serving: several resident scenes, render requests admitted by memory and   */
/* batched on the device in fixed-size tiles (continuous batching).           */
/* ------------------------------------------------------------------------- */
typedef struct gf_server_s* gf_server;

typedef struct {
    gf_scene scene;
    gf_camera camera;
    gf_render_desc render;
    float* out;          /* device width*height float32 radiance, caller-owned */
} gf_request;

/* mem_budget: bytes of device workspace the admitted requests may hold at
 * once (each request holds width*height*32 bytes of rays while in flight).
 * tile_rays: rays per tile; max_tiles: tiles per device batch.  The server
 * also allocates, once, the tracking workspace of one batch (at most
 * 3072 x 62 KB).  GF_ENOMEM / GF_EDEVICE if an allocation fails. */
gf_status gf_server_create(size_t mem_budget, int tile_rays, int max_tiles, void* stream, gf_server* out);
gf_status gf_server_destroy(gf_server server);
/* Queues a request (non-blocking); *id receives its id.  GF_EINVAL if it can
 * never fit the budget. */
gf_status gf_server_submit(gf_server server, const gf_request* req, uint64_t* id);
/* Advances the scheduler: admits queued requests (FIFO) while memory allows,
 * launches the next batch of tiles from the admitted requests, shortest
 * remaining work first (rays left x samples, multiple scattering counted 3x),
 * and retires requests whose tiles have all completed.  At most two batches
 * are in flight.  Non-blocking unless `wait` != 0. */
gf_status gf_server_step(gf_server server, int wait);
/* Retrieves up to max finished request ids (in completion order). */
gf_status gf_server_poll(gf_server server, uint64_t* ids, int max, int* n_done);
/* Requests queued, in flight, and device bytes currently held. */
gf_status gf_server_stats(gf_server server, int* queued, int* in_flight, size_t* bytes_held);
/* The server's scheduling policy on a virtual clock, without a device (the
 * serving workload: requests of uneven size admitted by memory and batched
 * as they arrive).  Request i (host arrays of n entries: width, height, spp,
 * multiple != 0) arrives at arrival_s[i] (sorted ascending).  Each step
 * retires the batches whose end has passed, admits queued requests in
 * arrival order while width*height*32 bytes (256 B aligned) fit a first-fit
 * pool of mem_budget bytes, and plans batches exactly as gf_server_step does
 * while fewer than two are in flight; a batch starts when the previous one
 * ends and takes sum over its tiles of rays x spp x (3 if multiple) divided
 * by work_per_s seconds.  Outputs (host, n): admit_s[i], done_s[i]; and the
 * largest number of pool bytes held at once (may be NULL).  GF_EINVAL for
 * invalid sizes, unsorted arrivals or a request larger than the budget. */
gf_status gf_server_simulate(size_t mem_budget, int tile_rays, int max_tiles, int64_t n, const int32_t* width,
                             const int32_t* height, const int32_t* spp, const int32_t* multiple,
                             const double* arrival_s, double work_per_s, double* admit_s, double* done_s,
                             size_t* max_held);

const char* gf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GABORFIELDS_H */
