/*
 * gaborfields.h - C ABI of the MI355X (gfx950) Gabor-field rendering library.
 *
 * The library traces rays through a volumetric density that is a mixture of
 * anisotropic Gabor kernels (paper: "Gabor Fields: Orientation-Selective
 * Level-of-Detail for Volume Rendering"; Sec. 3 for the extinction field,
 * optical depth and transmittance, Sec. 4.2 for the kernel, Sec. 4.4 for the
 * closed-form line integral, Sec. 4.5 for frequency / orientation masking,
 * Sec. 4.6 for the implementation details).
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
 *   and the ray-mask AND of Sec. 4.6 (implementation details).
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
    int majorant_grid;  /* resolution G of an optional majorant grid (G^3 voxels x 12 cells, the
                           point bound gf_density reports); 0 = none (the tracking kernels draw
                           their own per-ray majorants and do not use it) */
    float clamp_eps;    /* adaptive clamping (Sec. 4.4): each primitive's radius becomes min(r, E_i),
                           E_i^2 = 2 ln(rho |alpha_i| s_max / (2 pi s0 s1 s2 eps)) (0 when E_i^2 <= 0):
                           the Mahalanobis radius where the kernel's largest line integral across
                           it falls below eps (the carrier, |cos| <= 1, left out).  It changes the
                           density (a scene option).  0 = off. */
} gf_scene_desc;

typedef struct {
    uint64_t cells;            /* bit c keeps cell c (c = 3*level + bin); bits >= 12 ignored */
    const uint32_t* prim_bits; /* device, ceil(n/32) words, caller order; NULL = all */
    float lod_k;               /* continuous LOD cutoff (supplementary "LOD Selection"): a primitive is
                                  kept on a ray only when |f| d <= lod_k, d = |v| tc the distance from the
                                  ray origin to the primitive's Mahalanobis-closest point (kept when
                                  tc <= 0).  lod_k = R / (4 tan(fov/2)) puts the cutoff at the Nyquist
                                  frequency of an R-pixel camera.  0 = off.  In gf_render it applies to
                                  camera segments only. */
} gf_mask;

typedef struct {
    int64_t n;
    float rho, trunc_r, clamp_eps;
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
 * (Sec. 3, Eq. 3; accumulate-then-exponentiate as in Sec. 4.6 implementation
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
 * points: pts device n x 3; kappa, kbar device n (kbar may be NULL; it needs
 * a scene built with majorant_grid > 0). */
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

/* Per-segment stochastic mask strategies (Sec. 4.5.1 frequency levels,
 * Sec. 4.5.2 orientation bins; the two strategy tables of Appendix B).  A
 * segment draws four uniforms: u0 for its level strategy and u_l for the bin
 * strategy of each traced level l >= 1 (level 0, the low-pass level, has no
 * orientation and keeps all its bins).  The result is a weight per cell; a
 * primitive's density on the segment is multiplied by its cell's weight
 * (0: not traced).  Every stochastic strategy has expected weight 1 per cell,
 * so the segment's optical depth is unbiased; the threshold strategies drop
 * aligned bins deterministically.  P = 4 levels, K = 3 bins,
 * e = 1 - beta, x = u0^(1/e) a power-law draw:
 *   GF_LEVEL_ALL            every level, weight 1
 *   GF_LEVEL_UNIFORM        level floor(P u0), weight P
 *   GF_LEVEL_POWER          level floor(P x), weight 1 / (b^e - a^e) for its
 *                           bucket [a, b) = [l/P, (l+1)/P)
 *   GF_LEVEL_UNIFORM_CV     level 0 weight 1 (control variate) and one of the
 *                           levels 1..P-1 uniformly, weight P - 1
 *   GF_LEVEL_POWER_CV       level 0 weight 1 and level 1 + floor((P-1) x),
 *                           weight 1 / (b^e - a^e) over buckets of width 1/(P-1)
 *   GF_LEVEL_POWER_CV_ACCUM levels 0..floor(P x), level j with weight
 *                           1 / (1 - (j/P)^e)
 * With a_k = |v.e_k| / |v| the alignment of the segment with bin k's axis,
 * w_k = exp(-m_lk^2 a_k^2 / 2) (m_lk the cell's median |k_W|, k_W = S R^T 2 pi f)
 * and W = sum_k w_k:
 *   GF_BIN_ALL              every bin, weight 1
 *   GF_BIN_THRESHOLD        bins with a_k <= delta, weight 1 (threshold culling)
 *   GF_BIN_UNIFORM          bin floor(K u_l), weight K
 *   GF_BIN_IMPORTANCE       bin k with probability w_k / W, weight W / w_k
 *   GF_BIN_THRESHOLD_UNIFORM bins with a_k <= delta weight 1, plus one of the
 *                           N others uniformly, weight N
 *   GF_BIN_MIXTURE          (not in the paper) probability w_k/(2W) + 1/(2K),
 *                           weight its inverse (at most 2K): importance
 *                           sampling with bounded weights */
typedef enum {
    GF_LEVEL_ALL = 0,
    GF_LEVEL_UNIFORM = 1,
    GF_LEVEL_POWER = 2,
    GF_LEVEL_UNIFORM_CV = 3,
    GF_LEVEL_POWER_CV = 4,
    GF_LEVEL_POWER_CV_ACCUM = 5
} gf_level_strategy;

typedef enum {
    GF_BIN_ALL = 0,
    GF_BIN_THRESHOLD = 1,
    GF_BIN_UNIFORM = 2,
    GF_BIN_IMPORTANCE = 3,
    GF_BIN_THRESHOLD_UNIFORM = 4,
    GF_BIN_MIXTURE = 5
} gf_bin_strategy;

typedef struct {
    int spp;            /* camera samples per pixel / ray */
    int multiple;       /* 0: single scattering, 1: multiple scattering */
    int max_scatter;    /* multiple: a collision after this many scatterings ends the path with 0 */
    float albedo;       /* single-scattering albedo */
    float hg_g;         /* Henyey-Greenstein asymmetry (0 = isotropic) */
    float env;          /* constant environment radiance */
    int stochastic;     /* 1: every segment draws its own cell weights by the two strategies below,
                           applied on top of `mask` (Sec. 4.5.1-4.5.2) */
    int level_strategy; /* gf_level_strategy */
    int bin_strategy;   /* gf_bin_strategy */
    float beta;         /* power-law shape, 0 <= beta < 1 */
    float delta;        /* alignment threshold of the threshold strategies, in [0, 1] */
    int free_flight;    /* 0: weighted delta tracking, transmittances by ratio tracking;
                           1: CDF inversion of the closed-form optical depth (Sec. 3 and Sec. 4.4),
                           transmittances exp(-tau) from the closed form */
    int transmittance;  /* free_flight 0, single scattering: the shadow segment's transmittance by
                           0 ratio tracking, 1 the closed form exp(-tau) (Sec. 4.4; the tomography case
                           of Sec. 4.6); same mean, no variance.  free_flight 1 always uses 1.
                           With 1 in an image launch (image_width > 0) the shadow direction of a
                           sample is shared by the rays of an 8x8 pixel tile (drawn from the
                           tile's stream): each ray's estimate stays unbiased and the tile's
                           shadow rays trace as one packet; a ray list draws one per ray. */
    uint64_t shadow_cells; /* single scattering: cells the shadow rays trace, fixed (Zero-NEE of
                              Sec. 4.6 implementation details: shadow rays against the low-pass level,
                              cells 0x7); 0 = the shadow segment's own mask */
    gf_mask mask;       /* fixed mask; its lod_k applies to camera segments */
    uint64_t seed;
} gf_render_desc;

/* Radiance per ray (Sec. 3 radiative transfer with a constant environment).
 * Free flights: signed-weight delta tracking against the per-ray envelope
 * majorant of gf_transmittance_ratio, whose per-cell multipliers are the
 * cell weights capped at 18 (the estimators stay unbiased for any positive
 * majorant; weights above the cap only cost variance), with ratio-tracked
 * transmittances; or (free_flight = 1) the inverse of the cumulative
 * closed-form optical depth with exact transmittances.
 * Single: escape -> w env; real collision -> w albedo T(x, isotropic
 * direction) env.  Multiple: free flights with albedo and HG scattering until
 * escape; a collision after max_scatter scatterings ends the path with 0.
 * Outputs (device n, variances / T may be NULL): L mean / variance over spp,
 * primary-segment transmittance mean / variance.  image_width as for
 * gf_optical_depth.  Each sample of a ray is traced by one lane with random
 * streams keyed by (seed, ray index, sample), so in a ray list a ray's
 * result depends on its index but not on which rays are traced beside it.
 * In an image launch (image_width > 0) the shadow directions of single
 * scattering with closed-form transmittance come from the stream of the
 * ray's 8x8 pixel tile (seed, tile, sample), shared by the tile's rays:
 * every ray's estimate stays unbiased and the tile's shadow segments trace
 * as one packet; a tile's result then depends on the tile only.  The
 * samples of 64 rays may be spread over several work units (waves), their
 * values stored and summed in sample order afterwards: the result has the
 * same bits as one lane summing them.  The call allocates its tracking
 * workspace (and that per-sample storage) stream-ordered. */
gf_status gf_render_rays(gf_scene scene, const float* rays, int64_t n, int image_width, const gf_render_desc* desc,
                         float* L_mean, float* L_var, float* T_mean, float* T_var, void* stream);

/* Work of gf_render_rays with the same arguments (same random streams):
 * counts[0] tentative collisions, [1] internal LBVH nodes the kernel visited,
 * [2] primitive records it read at leaves, [3] windows, [4] tentative points
 * the estimators consume (all of a ratio-tracked segment's, a delta-tracked
 * one's up to its collision), and for those points [5] the internal nodes a
 * point query visits (box contains the point, cells pruned) and [6] the
 * primitives whose truncated support contains the point.  counts: device,
 * GF_RENDER_COUNTS x uint64, overwritten.  Used to count algorithmic bytes. */
#define GF_RENDER_COUNTS 7
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

/* Bytes of caller-owned device workspace gf_render needs for this camera and
 * description: the camera rays, the tracking lanes' state and, where the
 * render spreads each tile's samples over several work units, one L and one
 * T value per pixel and sample (at most 1 GiB; beyond that the samples of a
 * tile stay in one unit). */
gf_status gf_render_workspace_size(gf_scene scene, const gf_camera* cam, const gf_render_desc* desc,
                                   size_t* bytes);

/* Renders a camera image (the problem statement of Sec. 3: primitives, a
 * mask and rays in, radiance out), as gf_render_rays over the camera's rays
 * with the image width as tile width.  workspace: caller-owned device memory
 * of at least the size gf_render_workspace_size reports (256-byte aligned);
 * the call allocates nothing.  radiance: device height x width; primary_T:
 * device height x width or NULL (the camera segment's transmittance
 * estimate).  GF_EINVAL when ws_bytes is too small. */
gf_status gf_render(gf_scene scene, const gf_camera* cam, const gf_render_desc* desc, void* workspace,
                    size_t ws_bytes, float* radiance, float* primary_T, void* stream);

/* gf_render without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * file-scope device array of the library: the rays of up to 1,048,576
 * pixels, the tracking state of 1024 resident waves and 8,388,608 per-sample
 * values (pixels x spp x 2; a render that needs more keeps each tile's
 * samples in one work unit, which is slower on images with a few very
 * dense tiles), about 130 MB that each device the library runs on holds
 * until the process ends.  A camera with more pixels returns GF_EINVAL
 * before any launch.  Outputs as gf_render (radiance device height x width;
 * primary_T device height x width or NULL), bitwise the same.  Every call on one device shares the
 * array, which keeps the last call's contents: calls that overlap on one
 * device (other streams, other threads) race. */
gf_status gf_render_noalloc(gf_scene scene, const gf_camera* cam, const gf_render_desc* desc, float* radiance,
                            float* primary_T, void* stream);

/* Adjoint of gf_optical_depth (and of T = exp(-tau)): the gradient of a
 * rendered optical-depth / transmittance image with respect to every
 * primitive parameter, which the regression of Sec. 5 (differentiable
 * rendering of the kernel mixture) descends; here the closed-form segment
 * integral of Sec. 4.4 (Appendix A) is differentiated by hand, with the
 * chord-end (Leibniz) terms of the truncated support.  Accumulates
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
 * once (each request holds width*height*32 bytes of rays and
 * width*height*spp*4 bytes of per-sample radiance, each 256 B aligned,
 * while in flight).
 * tile_rays: rays per tile; max_tiles: tiles per device batch.  The server
 * also allocates, once, two batch slots, each with its own stream (default
 * priority) and tracking workspace (at most 3072 x 64 KB), so that a batch
 * starts while the previous one drains.  Ray generation runs on `stream`.
 * GF_ENOMEM / GF_EDEVICE if an allocation fails. */
gf_status gf_server_create(size_t mem_budget, int tile_rays, int max_tiles, void* stream, gf_server* out);
gf_status gf_server_destroy(gf_server server);
/* Queues a request (non-blocking); *id receives its id.  GF_EINVAL if it can
 * never fit the budget, or if max_tiles x tile_rays / 64 x spp reaches 2^30
 * (work units a batch indexes). */
gf_status gf_server_submit(gf_server server, const gf_request* req, uint64_t* id);
/* Advances the scheduler: admits queued requests (FIFO) while memory allows,
 * launches the next batch of tiles from the admitted requests, shortest
 * remaining work first (rays left x samples, multiple scattering counted 3x),
 * on a free batch slot, and retires requests whose tiles have all completed.
 * At most two batches are in flight, on the two slot streams, overlapping.
 * A batch's work units are single samples of 64 rays; each request's
 * samples are stored and averaged per ray in sample order when the batch
 * ends, so its image has the bits gf_render gives it.  The server renders
 * delta-tracked requests (free_flight 0).  Non-blocking unless `wait` != 0. */
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
 * arrival order while their pool bytes (as gf_server_create) fit a first-fit
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
