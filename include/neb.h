/*
 * neb.h -- C ABI of the Next Event Backtracking hot path on MI355X (gfx950).
 *
 * The operation follows the paper's statement of the problem (Jendersie,
 * "Next Event Backtracking", arXiv 1909.00573, Sec. 3): scene and lights
 * in, radiance image and NEE-vertex densities out.  One call of
 * neb_render runs the three passes of Sec. 3 once per iteration: view
 * paths with stored NEE vertices and emitter hits (Sec. 3.1), density,
 * NEE, photons traced from every NEE vertex and merged with view vertices
 * around each photon hit (Sec. 3.2), and weighted self emission (Sec. 3.3),
 * with the balance-heuristic weights of Sec. 4.  The density comes from the
 * lock-free sparse octree of Sec. 5 / Appendix B, whose surface is exported
 * separately (neb_octree_*).
 *
 * Conventions shared by every call:
 *  - every call returns neb_status; NEB_OK is 0.  Nothing throws or aborts
 *    across the ABI.  neb_last_error() returns a message for the last
 *    failure of the calling thread.
 *  - pointers marked "host" are read or written synchronously before the
 *    call returns; pointers marked "device" must be device memory of the
 *    current HIP device and are read or written in stream order on `stream`
 *    (a hipStream_t, NULL = the null stream).
 *  - the caller owns every buffer it passes in; the library owns everything
 *    it allocates internally and frees it in the matching destroy call.
 *  - a context or octree is not thread safe.
 *  - float layouts are little-endian, xyz (or rgb) interleaved.
 */
#ifndef NEB_H
#define NEB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NEB_OK = 0,
    NEB_ERR_INVALID_ARG = -1,   /* null pointer, size <= 0 or over a cap, NaN input */
    NEB_ERR_OUT_OF_MEMORY = -2, /* a device or host allocation failed */
    NEB_ERR_CAPACITY = -3,      /* a fixed pool is too small for the request */
    NEB_ERR_DEVICE = -4,        /* a HIP runtime call failed */
    NEB_ERR_STATE = -5          /* calls made in the wrong order */
} neb_status;

typedef struct neb_ctx_s* neb_ctx;
typedef struct neb_octree_s* neb_octree;

/* density providers for the flux conversion Phi = dE / rho (eq. flux) */
enum {
    NEB_DENSITY_OCTREE = 0,        /* one octree probe (Appendix B get_density) */
    NEB_DENSITY_OCTREE_ROBUST = 1, /* median of five probes (Appendix B, default) */
    NEB_DENSITY_MLP = 2,           /* learned density fitted to the robust octree, with octree
                                      fallback per region (see neb_configure_mlp) */
    NEB_DENSITY_ANALYTIC = 3,      /* test hook: rho0 + w * primary-hit density of the camera */
    NEB_DENSITY_RADIUS = 4,        /* fixed-radius count over the iteration's NEE vertices (the naive
                                      estimator Sec. 5 tried first): vertices within density_radius,
                                      over pi density_radius^2 */
    NEB_DENSITY_KNN = 5            /* k nearest neighbours over the iteration's NEE vertices (Sec. 5's
                                      second estimator): k / (pi d_k^2), d_k the distance to the k-th
                                      nearest vertex (a vertex at the query point counts); the mode-4
                                      estimate when fewer than k lie within density_radius */
};

/* neb_params.flags */
enum {
    NEB_FLAG_SINGLE_THREAD_OCTREE = 1, /* deposits by one GPU thread in (depth, pixel) order */
    NEB_FLAG_RECORD_PATHS = 2,         /* record the first iteration's view-path vertices */
    NEB_FLAG_NO_PHOTONS = 4            /* n_P = 0: path tracing with MIS over e and E only */
};

/* material types */
enum { NEB_MAT_LAMBERT = 0, NEB_MAT_MIRROR = 1, NEB_MAT_DIELECTRIC = 2, NEB_MAT_GGX = 3 };

typedef struct {
    int32_t width, height;     /* image size in pixels, 1 .. 8192 */
    int32_t max_path_len;      /* maximum path length in segments (camera = vertex 0), 1 .. 16 */
    int32_t octree_capacity;   /* child nodes, rounded up to whole blocks of 8, plus the root:
                                  1 + 8*ceil(n/8) nodes (Appendix B initialize), 1 .. 2^29 */
    float merge_radius;        /* r of the uniform merge kernel 1/(pi r^2), Sec. 3.2 */
    uint32_t seed, scene_id;   /* Philox-4x32-10 key (seed, scene_id) */
    int32_t density_mode;      /* NEB_DENSITY_* */
    float analytic_rho0;       /* NEB_DENSITY_ANALYTIC: constant term (per unit area, per iteration) */
    float analytic_cam_weight; /* NEB_DENSITY_ANALYTIC: weight of the camera's primary-hit density */
    int32_t flags;             /* NEB_FLAG_* */
    int32_t spp;               /* iterations this scene takes part in, counted from the last
                                  reset; 0 = every iteration (progressive) */
    int32_t light_photons;     /* n_LP: conventional light photons traced per iteration and merged
                                  with the view vertices (the optional technique of Sec. 4,
                                  eq. stdphotonpdf, weighted into eq. misw); 0 = none, at most
                                  2^26; not with NEB_DENSITY_MLP */
    float density_radius;      /* NEB_DENSITY_RADIUS, NEB_DENSITY_KNN: search radius (> 0) */
    int32_t knn_k;             /* NEB_DENSITY_KNN: k, 1 .. 16 */
    float nee_radius;          /* NEE recycling (Sec. 6, the subsection on reusing NEE events): > 0
                                  makes every vertex average the light samples of the NEE vertices
                                  within this radius (its own included), n_E of eq. misw being their
                                  number; 0 = off.  The same on/off for every scene of a batch; not
                                  with light_photons */
} neb_params;

/* Launch shapes of the traversal and photon kernels (neb_autotune picks
 * them; results do not depend on them).  Defaults: the shallowest stack
 * that holds every BVH, 8 resident closest-hit and 16 NEE blocks per CU
 * (at most as many as the LDS holds for the stack), 24 photon-merge blocks
 * per CU, queue order, concurrent. */
typedef struct {
    int32_t bvh_stack;            /* LDS traversal stack entries per lane: 32, 48 or 64; must
                                     exceed the entries every scene's BVH needs (a node visit
                                     pushes all but the nearest of its inner children) */
    int32_t trace_blocks_per_cu;  /* resident closest-hit blocks (one wave each) per compute unit;
                                     0 = one block per 64 queue slots, -1 = as many as the LDS holds;
                                     a launch never has more blocks than one per 64 queue slots */
    int32_t nee_blocks_per_cu;    /* resident NEE (shadow-ray) blocks per compute unit, same
                                     conventions */
    int32_t photon_blocks_per_cu; /* photon-merge blocks (one wave each) per compute unit, 0..64;
                                     0 = one block per 256 queue slots */
    int32_t photon_order;         /* 1: merge photons in the spatial (Morton) order of their hits,
                                     each XCD taking a contiguous share; 0: queue order */
    int32_t concurrent;           /* 1 (default): NEE's shadow rays and the merge grid run on a
                                     second stream beside the octree deposits and the density, each
                                     bounce's merges beside the next bounce's closest hits, and
                                     within one neb_render call each iteration but the last runs
                                     the next one's camera pass on a third stream; 0: every launch
                                     on the caller's stream, one after another */
} neb_launch_config;

/* One material per entry; emission is radiance leaving the front side of
 * the triangle (the side its counter-clockwise normal points to). */
typedef struct {
    int32_t type;        /* NEB_MAT_* */
    float albedo[3];     /* reflectance (Lambert, mirror, GGX) or transmittance tint (dielectric) */
    float ior;           /* dielectric index of refraction (outside is 1) */
    float alpha;         /* GGX roughness parameter, used as alpha directly */
    float emission[3];   /* radiance; an emitter with zero albedo ends paths */
} neb_material;

typedef struct {
    float pos[3];
    float power[3];      /* watts; isotropic point light of intensity power / (4 pi) */
} neb_point_light;

typedef struct {
    float eye[3], look_at[3], up[3];
    float vfov_deg;      /* vertical field of view of the pinhole camera */
} neb_camera;

typedef struct {
    /* photons: NEB photons emitted (visible NEE samples with rho > 0, eq. flux),
     * counted as they leave the virtual light, before their first scatter */
    int64_t iterations, paths, vertices, photons, photon_segments, merges, nee_visible, events, rays;
    /* octree: capacity, nodes allocated, depth, split failures, conserved ledger S
     * (sum of leaf counts - 4 * sum of the iteration of every allocated block),
     * counted deposits D (S == D whenever no deposit was lost), rejected
     * out-of-bounds deposits, deposits that gave up waiting for a split */
    int64_t oct_capacity, oct_allocated, oct_depth, oct_overflow, oct_ledger, oct_deposits,
        oct_rejected, oct_lost;
    /* work counters for algorithmic-byte accounting: photon states read by the
     * merge kernel (hits and misses), photon states written for the next
     * bounce, grid cells visited and view vertices tested by the merge gather */
    int64_t photon_items, photon_continued, grid_cells, candidates;
    /* rays = camera_rays + shadow_rays + photon rays */
    int64_t camera_rays, shadow_rays;
    /* BVH nodes fetched and triangles tested by all traversals */
    int64_t bvh_nodes, bvh_tris;
    /* conventional light photons emitted (their segments and merges are
     * counted with the NEB photons') */
    int64_t light_photons;
    /* bvh_nodes and bvh_tris split by the rays that did the work: camera
     * rays, photon rays (NEB and light photons), NEE shadow rays */
    int64_t bvh_nodes_camera, bvh_nodes_photon, bvh_nodes_shadow, bvh_tris_camera, bvh_tris_photon, bvh_tris_shadow;
} neb_stats;

/* per-kernel device time, collected with HIP events on the launch stream */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} neb_kernel_time;

/* view-path record of the first rendered iteration, one per (pixel, depth) */
typedef struct {
    int32_t type;   /* 0 none, 1 scatter, 2 specular reflection, 3 refraction,
                       4 path ended at this hit, 5 ray escaped at this depth */
    int32_t mat, prim;
    float pos[3];
} neb_path_record;

/* ---------------------------------------------------------------------- */
/* rendering context                                                       */
/* ---------------------------------------------------------------------- */

/* Validates the parameters and allocates, on the current device, the pools
 * of one iteration of the method's three passes (Sec. 3: the view-path
 * queues and the NEE-vertex store of pass 1, Sec. 3.1; the shadow rays and
 * photon queues of pass 2, Sec. 3.2; the emitter-hit events of pass 3,
 * Sec. 3.3), the merge grid of the photon merges (Sec. 4, eq. photonpdf),
 * the density octree's node pool (Sec. 5.1, 5.4) and the images.  The
 * context owns them until neb_destroy.  NEB_ERR_INVALID_ARG on bad
 * parameters, NEB_ERR_OUT_OF_MEMORY if the pools do not fit.  Same as
 * neb_create_batch(params, 1, out). */
neb_status neb_create(const neb_params* params, neb_ctx* out);

/* A context that renders n_scenes (1..256) independent scenes together:
 * every stage of an iteration (Sec. 3 passes 1-3) is one launch over all
 * scenes, which share the BVH pool (one tree per scene), the octree node
 * pool (scene s owns the 1 + 8*ceil(octree_capacity/8) nodes of params[s],
 * Sec. 5) and the queues.  params: n_scenes host entries; image size, path length, octree
 * capacity, merge radius, RNG key, analytic density terms and spp may
 * differ per scene; density_mode and flags must be equal (else
 * NEB_ERR_INVALID_ARG).  A scene takes part in iterations 1..spp (all if
 * spp is 0); its paths and photons use its own key and scene-local pixel
 * numbers, so it renders the same estimator as alone.  Path records of a
 * batch are indexed by the pixel numbered over all scenes in order. */
neb_status neb_create_batch(const neb_params* params, int32_t n_scenes, neb_ctx* out);
/* Deep-copies the scene (host arrays) into library-owned device memory,
 * builds the BVH and the light table (emissive triangles and point lights,
 * selected in proportion to power), and initialises the octree over the
 * bounding box of the vertices (Appendix B initialize).  Clears the image
 * and the iteration counter.  vertices: nv*3 floats; tris: nt*3 indices;
 * tri_material: nt material indices; materials: nm entries; point_lights:
 * npl entries (may be NULL when npl == 0); camera: one entry.
 * NEB_ERR_INVALID_ARG on out-of-range indices, NaN coordinates, a flat
 * bounding box or a scene without lights. */
neb_status neb_set_scene(neb_ctx ctx, const float* vertices, int32_t nv, const int32_t* tris,
                         const int32_t* tri_material, int32_t nt, const neb_material* materials,
                         int32_t nm, const neb_point_light* point_lights, int32_t npl,
                         const neb_camera* camera);

/* neb_set_scene for scene `scene` of a batch (arguments as above; at most
 * 65536 materials over the batch).  The host copy is validated and its BVH
 * built here; the pools are uploaded by the next neb_render, neb_reset or
 * neb_autotune once every scene is set.  Setting a scene restarts the
 * progression of every scene of the context.  NEB_ERR_STATE from neb_set_scene
 * on a context of more than one scene. */
neb_status neb_set_batch_scene(neb_ctx ctx, int32_t scene, const float* vertices, int32_t nv,
                               const int32_t* tris, const int32_t* tri_material, int32_t nt,
                               const neb_material* materials, int32_t nm,
                               const neb_point_light* point_lights, int32_t npl,
                               const neb_camera* camera);

/* Runs n_iterations progressive iterations (one sample per pixel each) on
 * `stream`, continuing from the context's iteration counter; the octree
 * integrates its counts over the iterations (Sec. 5.3, time integration).
 * Work forked onto the library's own streams is joined back into `stream`
 * before the last iteration ends, so nothing is in flight between calls and
 * the result does not depend on how the iterations are split over calls.
 * Returns after enqueueing; NEB_ERR_STATE unless every scene is set. */
neb_status neb_render(neb_ctx ctx, int32_t n_iterations, void* stream);

/* mode 1: neb_render replays one captured iteration per iteration (a HIP
 * graph, captured on first use) instead of launching its kernels one by
 * one; mode 2: each neb_render call is one launch of a graph that holds
 * the whole call (its iterations, and the camera passes forked beside
 * them, exactly as the eager launches order them; captured on the first
 * call with that iteration count, the graphs of the last four counts are
 * kept); mode 0: eager launches (the default).  The results are those of
 * the eager launches; calls or iterations that record paths or kernel
 * times, and the learned density's iterations, are always launched
 * eagerly.  NEB_ERR_INVALID_ARG for another mode. */
neb_status neb_use_graph(neb_ctx ctx, int32_t mode);

/* Times trial_iterations (1..64) real iterations of the context for each
 * candidate launch shape — traversal stack depth and closest-hit blocks per
 * CU, then NEE blocks per CU, then the photon stage (order and merge grid),
 * each by the time of its own kernels; then the photon order and the
 * closest-hit and merge blocks per CU once more by the time of whole
 * iterations with the launches as they run (beside each other, the shape
 * fastest alone is not the iteration's) — keeps the fastest, writes it to
 * *chosen (may be NULL) and resets the context as neb_reset does.
 * Synchronises `stream`. */
neb_status neb_autotune(neb_ctx ctx, int32_t trial_iterations, void* stream, neb_launch_config* chosen);

/* Sets or reads the launch shapes (NEB_ERR_INVALID_ARG out of range,
 * NEB_ERR_CAPACITY if the stack is not deeper than a scene's BVH needs). */
neb_status neb_set_launch_config(neb_ctx ctx, const neb_launch_config* cfg);
neb_status neb_get_launch_config(neb_ctx ctx, neb_launch_config* cfg);

/* Mean radiance over the rendered iterations, height*width*3 floats,
 * row-major from the top-left pixel: the progressive estimate of the
 * method, each iteration's random hits (e), NEE (E), NEB photon merges (P)
 * and light-photon merges (LP) combined with the balance heuristic
 * (Sec. 4, eq. misweight over the techniques of eq. misw).  rgb is
 * device memory if is_device_ptr, else host memory (then the call
 * synchronises); the caller owns it.  NEB_ERR_STATE before the first
 * neb_set_scene. */
neb_status neb_get_image(neb_ctx ctx, float* rgb, int32_t is_device_ptr, void* stream);

/* neb_get_image for scene `scene` of a batch: its own height*width*3
 * floats, averaged over the iterations it took part in.  neb_get_image is
 * scene 0.  NEB_ERR_STATE before the pools are uploaded. */
neb_status neb_get_scene_image(neb_ctx ctx, int32_t scene, float* rgb, int32_t is_device_ptr,
                               void* stream);

/* Mean radiance split by technique: random hits (e), NEE (E) and NEB photon
 * merges (P), each height*width*3 floats; any pointer may be NULL. */
neb_status neb_get_technique_images(neb_ctx ctx, float* e, float* E, float* P, int32_t is_device_ptr,
                                    void* stream);
neb_status neb_get_scene_technique_images(neb_ctx ctx, int32_t scene, float* e, float* E, float* P,
                                          int32_t is_device_ptr, void* stream);

/* The two alternative density providers on a point set (Sec. 5): the
 * density of n_query points over n points, per unit area, by
 * NEB_DENSITY_RADIUS (mode 4) or NEB_DENSITY_KNN (mode 5) with the given
 * radius and k, exactly as a render computes them over its NEE vertices.
 * points: n*3 floats, queries: n_query*3 floats, out: n_query floats, all
 * device memory on the current device; stream-ordered (the call allocates
 * and frees a temporary grid, and returns after the work is done).
 * n may be 0 (all densities 0).  NEB_ERR_INVALID_ARG for a bad mode,
 * radius or k, or negative sizes. */
neb_status neb_point_density(const float* points, int32_t n, const float* queries, int32_t n_query, int32_t mode,
                             float radius, int32_t k, float* out, void* stream);

/* neb_point_density for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and results; it calls no hipMalloc, hipFree or
 * allocating library routine and does not synchronise: the work is enqueued
 * on `stream` and the call returns.  The grid lives in a fixed device array
 * of the library (about 10.5 MB on every device it runs on, held until the
 * process ends), so n is at most 524288 (2^19) points (NEB_ERR_CAPACITY
 * beyond); n_query is not limited (queries and out are the caller's).  Every
 * call on one device shares that array and rewrites all of it that it uses
 * (the bucket counts are cleared by a kernel at the start of each call):
 * calls that overlap on one device, e.g. on two streams without ordering,
 * race and give wrong results. */
neb_status neb_point_density_noalloc(const float* points, int32_t n, const float* queries, int32_t n_query,
                                     int32_t mode, float radius, int32_t k, float* out, void* stream);

/* Mean radiance of the conventional light-photon merges (LP, Sec. 4,
 * eq. stdphotonpdf) of scene `scene`: height*width*3 floats, zero when the
 * scene traces no light photons.  The image of neb_get_scene_image is the
 * sum of e, E, P and LP.  LP is device memory if is_device_ptr, else host
 * memory (then the call synchronises). */
neb_status neb_get_scene_light_photon_image(neb_ctx ctx, int32_t scene, float* LP, int32_t is_device_ptr,
                                            void* stream);

/* Density of NEE vertices at n surface points from the context's octree in
 * its current state: the robust query of Appendix B (get_density_robust:
 * the median of five probes, the point and four offsets along tangents
 * taken from the normal), each probe the count of the leaf it lands in
 * over the area of the surface's plane inside that leaf's box (Sec. 5.3,
 * eq. octdensity, the area by eq. area and Appendix A), scaled to one
 * iteration.  pos, nrm: n*3 floats; out: n floats; all device memory if
 * is_device_ptr, else host memory (then the call synchronises).
 * NEB_ERR_INVALID_ARG for n < 0 or a null pointer, NEB_ERR_STATE before
 * the scene is set. */
neb_status neb_query_density(neb_ctx ctx, const float* pos, const float* nrm, int32_t n, float* out,
                             int32_t is_device_ptr, void* stream);

/* Counters accumulated since the last reset, over all scenes of the
 * context: the work of the passes of Sec. 3 (paths, NEE vertices, shadow
 * rays, photons and their segments, merge candidates and accepted merges,
 * traversal fetches) and the state of the density octrees of Sec. 5
 * (nodes, depth, the Appendix B insert ledger; fields summed over the
 * scenes' octrees, depth the deepest).  out: host memory, owned by the
 * caller.  Synchronises the context's last stream. */
neb_status neb_get_stats(neb_ctx ctx, neb_stats* out);

/* Copies the path records of the first rendered iteration to host memory:
 * width*height*max_path_len records (pixel-major).  NEB_ERR_STATE unless the
 * context was created with NEB_FLAG_RECORD_PATHS and has rendered. */
neb_status neb_get_path_records(neb_ctx ctx, neb_path_record* out, int64_t n);

/* Exports the context's octree node array (host, up to cap entries) and
 * its info (see neb_octree_export); scene 0 of a batch.  The scene variant
 * exports the octree of scene `scene` (node links are pool indices: a
 * child pointer -v of a node in the export is word v - root, where root is
 * the sum of the rounded capacities of the scenes before it). */
neb_status neb_get_octree(neb_ctx ctx, int32_t* nodes, int32_t cap, int64_t info[8]);
neb_status neb_get_scene_octree(neb_ctx ctx, int32_t scene, int32_t* nodes, int32_t cap,
                                int64_t info[8]);

/* enable != 0 starts recording a HIP event pair around every kernel launch
 * of this context (clearing earlier records); 0 stops.  Recording adds a
 * few microseconds per launch. */
neb_status neb_profile_kernels(neb_ctx ctx, int32_t enable);

/* Per-kernel totals recorded so far (host array of cap entries, *n_out set
 * to the number of kernels written).  Synchronises the recorded events. */
neb_status neb_get_kernel_profile(neb_ctx ctx, neb_kernel_time* out, int32_t cap, int32_t* n_out);

/* Clears the images, the statistics, every octree and the iteration
 * counter (uploads the pools first if the scenes changed). */
neb_status neb_reset(neb_ctx ctx);

void neb_destroy(neb_ctx ctx);
const char* neb_status_string(neb_status s);
const char* neb_last_error(void);

/* ---------------------------------------------------------------------- */
/* learned density (stands in for the octree query of Sec. 5 / eq.         */
/* octdensity; the model is not in the paper)                              */
/* ---------------------------------------------------------------------- */

/* Model: 80 encoded inputs (the point normalised to the octree box, q in
 * [0,1)^3, the unit normal n, then sin and cos of 2^f pi c for the six
 * coordinates c = q0,q1,q2,n0,n1,n2 and octaves f = 0..5, feature
 * 6 + 12 c + 2 f, then two zeros) -> 64 -> 64 -> 64 (ReLU) -> 1 output y;
 * log rho = mu + sigma * y.  Hidden layers run on the matrix cores with
 * bf16 operands and FP32 accumulation; the parameters are FP32 master
 * copies trained with Adam on the mean squared error of y against
 * (log rho_target - mu) / sigma.  Flat parameter layout (host and device):
 * W1 (80 x 64, row k = input feature k), b1 (64), W2 (64 x 64), b2,
 * W3 (64 x 64), b3, w4 (64), b4 (1). */
#define NEB_MLP_PARAMS 13569

typedef struct neb_mlp_s* neb_mlp;

/* Settings of NEB_DENSITY_MLP.  The model stands in for the octree's
 * density query (Sec. 5.3, eq. octdensity, and the five-probe median of
 * Appendix B, get_density_robust), which stays the judge and the fallback.
 * The first train_iterations iterations use the robust octree; after each,
 * the NEE vertices with rho > 0 become the training pool (position, normal,
 * log rho) and steps_per_iteration (0 allowed) Adam steps are taken on
 * batches of `batch` draws from it (mu, sigma are the first pool's mean and
 * standard deviation unless a model was given with neb_set_mlp_model).
 * Later iterations take rho from the model; the octree stops counting (it
 * keeps the density of the training iterations) and judges the model:
 * every vertex of the first model iteration, then, every probe_every
 * iterations, each vertex with probability probes / (vertices of the
 * iteration) (its own draw from the probe stream, counter (pixel,
 * iteration, depth)), is compared with the robust octree query.  A probe is
 * over the bound when |rho_model - rho_octree| > max_rel_error * rho_octree
 * (or rho_octree = 0 < rho_model).  Each of the 32^3 regions of the octree
 * box keeps the model while the model's densities summed over the region's
 * probes so far are within max_rel_error of the octree's summed over the
 * same probes (the model's bias in the region; the octree's per-cell
 * counting noise, larger than a 10 % bound probe by probe, averages out
 * there), else its vertices take the octree query.  The status reports the
 * probes of the regions that keep the model and how many of them are over
 * the bound one by one. */
typedef struct {
    int32_t train_iterations;    /* default 4 */
    int32_t steps_per_iteration; /* default 250 */
    int32_t batch;               /* default 65536, 16 .. 1048576 */
    float lr, beta1, beta2, eps; /* default 2e-3, 0.9, 0.999, 1e-8 */
    int32_t probe_every;         /* default 8 */
    int32_t probes;              /* default 4096 */
    float max_rel_error;         /* default 0.1 */
    uint32_t seed;               /* initial weights (He uniform) and batch draws */
} neb_mlp_params;

typedef struct {
    int32_t phase;               /* 0 training on the octree, 1 model in use */
    int64_t adam_steps;
    double last_loss;            /* mean loss over the last training iteration's steps */
    float mu, sigma;
    int64_t probes, probes_bad;  /* probe comparisons so far, and those over the bound */
    int64_t regions_probed, regions_disabled;
    int64_t fallback_queries;    /* vertex densities taken from the octree in model iterations */
    /* probes so far in the regions that keep the model, and those of them
     * over the bound: their ratio estimates the fraction of model-served
     * densities whose error exceeds max_rel_error */
    int64_t probes_served, probes_served_bad;
} neb_mlp_status;

/* Sets the model settings of a context created with NEB_DENSITY_MLP (one
 * scene) and restarts it (NULL = defaults).  NEB_ERR_STATE for other
 * contexts, NEB_ERR_INVALID_ARG for values out of range. */
neb_status neb_configure_mlp(neb_ctx ctx, const neb_mlp_params* params);
neb_status neb_get_mlp_status(neb_ctx ctx, neb_mlp_status* out);
/* Gives the context a model (params: host, NEB_MLP_PARAMS floats in the
 * flat layout below; log rho = mu + sigma * y) in place of the seeded
 * initial weights, and restarts it.  The training iterations still fill the
 * octree and take steps_per_iteration Adam steps from these weights (none
 * with 0); mu and sigma are kept.  params == NULL returns to the seeded
 * initial weights.  NEB_ERR_STATE for contexts without NEB_DENSITY_MLP,
 * NEB_ERR_INVALID_ARG for non-finite values or sigma <= 0. */
neb_status neb_set_mlp_model(neb_ctx ctx, const float* params, float mu, float sigma);
/* The region gates (32^3 host int32 each; any may be NULL): gate[r] = 1
 * while region r keeps the model, probes[r] and bad[r] its probe tallies.
 * Region r = x + 32 (y + 32 z) of the cell (x, y, z) of the octree box cut
 * 32 times per axis.  Synchronises the context's stream. */
neb_status neb_get_mlp_gates(neb_ctx ctx, int32_t* gate, int32_t* probes, int32_t* bad);
/* The context's model parameters (host, NEB_MLP_PARAMS floats). */
neb_status neb_get_mlp_weights(neb_ctx ctx, float* params);

/* A standalone model for batches of up to max_batch samples.  init: host,
 * NEB_MLP_PARAMS floats, or NULL for He-uniform weights from `seed` and
 * zero biases; mu = 0, sigma = 1. */
neb_status neb_mlp_create(const float* init, uint32_t seed, int32_t max_batch, neb_mlp* out);
neb_status neb_mlp_set_normalization(neb_mlp mlp, float mu, float sigma, void* stream);
/* log rho at n points: q, nrm device (n*3 floats; q normalised to
 * [0,1)^3), out device (n floats). */
neb_status neb_mlp_infer(neb_mlp mlp, const float* q, const float* nrm, int32_t n, float* out, void* stream);
/* Gradient of the batch's mean loss (device q, nrm: n*3 floats; log_rho:
 * n floats; 1 <= n <= max_batch) into grad (device, NEB_MLP_PARAMS floats)
 * and the loss into *loss (host; the call synchronises `stream`). */
neb_status neb_mlp_gradient(neb_mlp mlp, const float* q, const float* nrm, const float* log_rho, int32_t n,
                            float* grad, float* loss, void* stream);
/* One Adam step on the batch's gradient. */
neb_status neb_mlp_train_step(neb_mlp mlp, const float* q, const float* nrm, const float* log_rho, int32_t n,
                              float lr, float beta1, float beta2, float eps, void* stream);
neb_status neb_mlp_get_params(neb_mlp mlp, float* params);
void neb_mlp_destroy(neb_mlp mlp);

/* ---------------------------------------------------------------------- */
/* density octree (Sec. 5, Appendix B), batched and stream-ordered         */
/* ---------------------------------------------------------------------- */

/* Octree over [scene_min, scene_max] (host, 3 floats each; enlarged by 0.1 %
 * per side as in Appendix B initialize) holding the root and `capacity`
 * child nodes rounded up to whole blocks of 8 (1 + 8*ceil(capacity/8)
 * nodes).  The root starts as an empty leaf; iteration 1 is set. */
neb_status neb_octree_create(const float scene_min[3], const float scene_max[3], int32_t capacity,
                             neb_octree* out);

/* Sets the iteration (Appendix B set_iteration): split threshold
 * 4*min(iter,1000), density scale 1/min(iter,1000), filling stops after
 * iteration 1000.  Iterations must not decrease (NEB_ERR_STATE) unless the
 * counters were cleared. */
neb_status neb_octree_set_iteration(neb_octree oct, int32_t iter);

/* Deposits n points (device, n*3 floats) with lock-free counter
 * increments, compare-and-swap counting and on-the-fly splits (Sec. 5.1,
 * 5.2).  single_thread != 0 makes one GPU thread insert them in array
 * order (deterministic; equals a sequential insertion). */
neb_status neb_octree_increment(neb_octree oct, const float* pos, int32_t n, int32_t single_thread,
                                void* stream);

/* Densities rho = c / |cell cap tangent plane| (eq. octdensity, eq. area)
 * at n points with normals (device, n*3 floats each) into out (device, n
 * floats); robust != 0 selects the five-probe median of Appendix B. */
neb_status neb_octree_density(neb_octree oct, const float* pos, const float* nrm, int32_t n,
                              int32_t robust, float* out, void* stream);

/* Zeroes every counter, keeps the child pointers (Appendix B clear_counters). */
neb_status neb_octree_clear_counters(neb_octree oct, void* stream);

/* Copies up to cap nodes to host memory (may be NULL) and fills info with:
 * capacity, allocated nodes, depth, ledger S, deposits D, split failures,
 * rejected deposits, lost deposits.  Synchronises `stream`. */
neb_status neb_octree_export(neb_octree oct, int32_t* nodes, int32_t cap, int64_t info[8], void* stream);

void neb_octree_destroy(neb_octree oct);

/* ---------------------------------------------------------------------- */
/* measurement                                                             */
/* ---------------------------------------------------------------------- */

/* Device-scope atomic throughput, the ceiling of the octree's lock-free
 * counting (Sec. 5.1, 5.2): blocks x 256 threads each make `ops`
 * increments of words picked by a hash of (thread, k) among n_words words
 * spaced `stride` ints apart; kind 0: returning atomic add, kind 1: a
 * compare-and-swap loop (load, CAS old -> old + 1 until it succeeds).
 * words: device, at least n_words * stride ints (the caller's, counts
 * accumulate); sink: device, blocks * 256 ints (each thread's fold of the
 * returned values).  Enqueued on `stream`; the caller times it.
 * NEB_ERR_INVALID_ARG for null pointers, sizes < 1 or kind out of range. */
neb_status neb_atomic_probe(int32_t* words, int32_t n_words, int32_t stride, int32_t blocks, int32_t ops,
                            int32_t kind, int32_t* sink, void* stream);

/* Random-access read throughput, the ceiling of the photon merges' lookups
 * (Sec. 3.2: each photon hit reads the cell table, candidate runs and merge
 * records of the view vertices near it): blocks x 256 threads each read
 * `ops` records of `width` 16-byte words (1 or 4: 16 or 64 bytes, aligned
 * to their size) at indices picked by a hash of (thread, k) among the
 * n_words 16-byte words of buf, eight reads in flight per thread.  buf:
 * device, n_words * 16 bytes (the caller's, only read); sink: device,
 * blocks * 256 floats (each thread's sum of what it read).  Enqueued on
 * `stream`; the caller times it.  NEB_ERR_INVALID_ARG for null pointers,
 * n_words < 4, width not 1 or 4, blocks or ops < 1. */
neb_status neb_gather_probe(const float* buf, int64_t n_words, int32_t width, int32_t blocks, int32_t ops,
                            float* sink, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NEB_H */
