/*
 * neb_oracle.c -- plain, slow FP64 reference of the Next Event Backtracking
 * estimator (Jendersie, "Next Event Backtracking", arXiv 1909.00573).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that the tests, the smoke check and the
 * bench's CPU baseline can compare the GPU library against an independent,
 * obviously correct implementation.  It shares no code, header, table or
 * constant generator with the GPU library.
 *
 * What follows the paper, and where:
 *   - three-pass algorithm: Sec. 3 (outline list and Fig. "algorithm"):
 *     pass 1 traces view paths and stores NEE vertices and random emitter
 *     hits (Sec. 3.1); pass 2 estimates the vertex density, computes NEE
 *     and traces photons from every NEE vertex, merging them with view
 *     vertices found around each photon hit (Sec. 3.2); pass 3 weights the
 *     stored emitter hits (Sec. 3.3).
 *   - flux of a virtual light: Phi = dE / rho, eq. (flux).
 *   - NEE contribution L_E, photon contribution L_P with the uniform
 *     kernel 1/(pi r^2), self emission L_e: Sec. 3.2 and 3.3.
 *   - MIS: balance heuristic eq. (misweight) with the path densities of
 *     eq. (rhpdf), (neepdf), (photonpdf) summed as in eq. (misw); here
 *     evaluated as EXPLICIT products over the whole path (no recursion).
 *   - optional conventional light photons (Sec. 4, eq. stdphotonpdf and
 *     the n_LP sum of eq. misw): n_LP photons per iteration, emitted from
 *     a light picked by power, merged at every non-delta hit with the view
 *     vertices within r (paths of length k + j for a view vertex of depth
 *     k and a photon of j segments).
 *   - density octree: Sec. 5.1 (counting), 5.2 (split, children start at
 *     parent/4), 5.3 (rho = c / |B cap P|, eq. octdensity), time
 *     integration (threshold and scale follow the iteration count), 5.4
 *     (sign-encoded child index, threshold 4), and the class of Appendix B
 *     (its initialisation, the 1000-iteration fill limit, the minimum-area
 *     clamp and the five-probe robust query with the upper median).
 *   - NEE recycling (Sec. 6): every vertex averages the light samples of
 *     the NEE vertices within a radius, n_E of eq. misw being their number.
 *   - the two estimators Sec. 5 tried before the octree, over the
 *     iteration's NEE vertices: the fixed-radius count (naive estimator)
 *     and the k-nearest-neighbour estimate (k >= 4), both by brute force.
 *   - the plane-box area is NOT evaluated with eq. (area); the oracle uses
 *     the plain definition: the area of the convex polygon obtained by
 *     clipping the plane with the box (the GPU uses eq. (area)).
 *
 * Readings where the paper is silent:
 *   - the octree counts NEE (view) vertices; later photon hits are merged
 *     against view vertices, never deposited.
 *   - concurrent-split semantics: a split that cannot allocate marks the
 *     leaf "split failed" (bit 30) and it keeps counting; deposits are
 *     never lost; the conserved ledger S = sum(leaf counts) -
 *     4 * sum(iteration of each allocated block) equals the number of
 *     counted deposits.  Nodes at depth 20 never split.
 *   - children get the current iteration as their start count at the
 *     moment of the split (equivalent to the prefill of unused nodes).
 *   - deposits are made after pass 1 in (depth, pixel) order.
 *   - path length counts segments, camera is vertex 0; a merge of a photon
 *     with j segments at a view vertex of depth k forms a path of length
 *     k + j + 1, which must not exceed the maximum.
 *   - NEE vertices are all view vertices of depth 1 .. maxlen-1 on
 *     non-black surfaces, delta surfaces included (no NEE contribution
 *     there, but they emit photons); occluded NEEs emit no photon.
 *   - delta BSDF pdfs are the discrete lobe probabilities.
 *   - no Russian roulette; geometric normals only; no eta^2 scaling.
 *   - NEE recycling borrows a neighbour's visibility and light point; the
 *     neighbour's own sample counts although it may be occluded from the
 *     receiver; not combined with light photons.
 *   - light photons: area lights emit with the cosine lobe around their
 *     normal, point lights uniformly over the sphere; the light vertex of
 *     their paths is the sampled light point; the density rho_{L-1} that
 *     their paths' NEB technique needs is queried at the photon's first
 *     hit (with that hit's normal), also when the merge happens there.
 *   - uniform random numbers are (x >> 8) * 2^-24 of Philox-4x32-10
 *     outputs, counter (pixel, iteration, depth, stream), key (seed,
 *     scene id); photon streams use counter (origin pixel, iteration,
 *     16 * origin depth + photon bounce, PHOTON); light photon i draws
 *     its light point with (i, iteration, 0, LIGHT), its direction with
 *     (i, iteration, 1, LIGHT) and its scattering after hit j with
 *     (i, iteration, j - 1, PHOTON).
 *
 * Precision: FP64 everywhere except the octree's cell addressing, which
 * follows the FP32 arithmetic of the class in Appendix B exactly (build
 * this file with -ffp-contract=off) so that a shared float deposit stream
 * yields the same tree as any other faithful implementation.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
typedef struct { double x, y, z; } v3;
static inline v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static inline v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static inline v3 hmul(v3 a, v3 b) { return mk(a.x * b.x, a.y * b.y, a.z * b.z); }
static inline double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 cross(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline double len(v3 a) { return sqrt(dot(a, a)); }
static inline v3 nrm(v3 a) { return scl(a, 1.0 / len(a)); }
static inline double maxc(v3 a) { return fmax(a.x, fmax(a.y, a.z)); }
static inline int is_zero(v3 a) { return a.x == 0.0 && a.y == 0.0 && a.z == 0.0; }
static inline v3 from_f(const float* f) { return mk(f[0], f[1], f[2]); }
static inline double comp(v3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

/* ------------------------------------------------------------------ */
/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                   */
/* ------------------------------------------------------------------ */
enum { TAG_CAMERA = 1, TAG_BSDF = 2, TAG_NEE = 3, TAG_PHOTON = 4, TAG_LIGHT = 7 };

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t n0 = hi_b ^ c1 ^ k0;
        uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0; c1 = lo_b; c2 = n2; c3 = lo_a;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

typedef struct { uint32_t key[2]; } rng_key;

static void uniforms(rng_key k, uint32_t a, uint32_t b, uint32_t c, uint32_t tag, double u[4]) {
    uint32_t ctr[4] = {a, b, c, tag}, out[4];
    orc_philox4x32_10(ctr, k.key, out);
    for (int i = 0; i < 4; ++i) u[i] = (double)(out[i] >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------ */
/* inputs (same memory layout as the Python input generator)          */
/* ------------------------------------------------------------------ */
typedef struct { int32_t type; float albedo[3]; float ior; float alpha; float emission[3]; } o_material;
typedef struct { float pos[3]; float power[3]; } o_point_light;
typedef struct { float eye[3], look_at[3], up[3], vfov_deg; } o_camera;

enum { M_LAMBERT = 0, M_MIRROR = 1, M_DIELECTRIC = 2, M_GGX = 3 };

typedef struct {
    int32_t width, height, max_path_len, octree_capacity;
    double merge_radius;
    uint64_t seed;
    uint32_t scene_id;
    int32_t density_mode;          /* 0 octree single probe, 1 octree robust, 3 analytic,
                                      4 fixed radius, 5 k nearest neighbours */
    double analytic_rho0, analytic_cam_weight;
    int32_t enable_photons;        /* 0: n_P = 0 (plain PT with MIS over e and E) */
    int32_t win_x0, win_y0, win_x1, win_y1;   /* pixel window, exclusive end; 0,0,0,0 = all */
    int32_t n_threads;
    int32_t record_paths;          /* record vertex sequences of the first iteration */
    int32_t light_photons;         /* n_LP: conventional light photons per iteration (0 = none) */
    double density_radius;         /* R of the fixed-radius and nearest-neighbour providers (modes 4, 5) */
    int32_t knn_k;                 /* k of the nearest-neighbour provider (mode 5) */
    double nee_radius;             /* NEE recycling radius (0 = each vertex uses its own NEE only) */
    /* learned-density runs: after iteration freeze_after (0 = never) the
     * octree takes no deposits and keeps the scalars of that iteration */
    int32_t freeze_after;
    /* optional density hook, called once per iteration after the densities
     * of pass 2 (a) with every NEE vertex of the iteration in canonical
     * order: position, normal, pixel, depth, and rho (in: the provider's
     * value, out: the value the iteration uses) */
    void (*density_hook)(int32_t n, const double* pos, const double* nrm, const int32_t* pixel,
                         const int32_t* depth, int32_t iter, double* rho);
} o_params;

typedef struct {
    double paths, vertices, photons, photon_segments, merges, nee_visible, events, rays;
    int64_t oct_nodes, oct_depth, oct_overflow, oct_ledger, oct_deposits, oct_capacity, oct_rejected;
    double light_photons;          /* light photons emitted */
} o_stats;

/* path record entry (first iteration only): one per (path, depth) */
typedef struct { int32_t type; int32_t mat; int32_t prim; float pos[3]; } o_record;
enum { EV_NONE = 0, EV_SCATTER = 1, EV_REFLECT = 2, EV_REFRACT = 3, EV_STOP = 4, EV_ESCAPE = 5 };

/* ------------------------------------------------------------------ */
/* plane-box intersection area: clip the plane with the box            */
/* ------------------------------------------------------------------ */
static int cmp_angle(const void* a, const void* b) {
    double x = ((const double*)a)[3], y = ((const double*)b)[3];
    return (x > y) - (x < y);
}

double orc_exact_area(const double bmin[3], const double bmax[3], const double p[3], const double n[3]) {
    v3 P = mk(p[0], p[1], p[2]);
    v3 N = nrm(mk(n[0], n[1], n[2]));
    v3 c[8];
    for (int i = 0; i < 8; ++i)
        c[i] = mk((i & 1) ? bmax[0] : bmin[0], (i & 2) ? bmax[1] : bmin[1], (i & 4) ? bmax[2] : bmin[2]);
    double s[8];
    for (int i = 0; i < 8; ++i) s[i] = dot(N, sub(c[i], P));
    double pts[24][4];
    int np = 0;
    for (int i = 0; i < 8; ++i)
        for (int ax = 0; ax < 3; ++ax) {
            int j = i | (1 << ax);
            if (j == i) continue;             /* each edge once: from the lower corner */
            v3 q;
            int have = 0;
            if (s[i] == 0.0) { q = c[i]; have = 1; }
            if (s[j] == 0.0) {
                if (have && np < 24) { pts[np][0] = q.x; pts[np][1] = q.y; pts[np][2] = q.z; ++np; }
                q = c[j]; have = 1;
            } else if (s[i] != 0.0 && ((s[i] < 0.0) != (s[j] < 0.0))) {
                double t = s[i] / (s[i] - s[j]);
                q = add(c[i], scl(sub(c[j], c[i]), t));
                have = 1;
            }
            if (have && np < 24) { pts[np][0] = q.x; pts[np][1] = q.y; pts[np][2] = q.z; ++np; }
        }
    double diag = len(sub(c[7], c[0]));
    /* remove duplicates */
    int m = 0;
    for (int i = 0; i < np; ++i) {
        int dup = 0;
        for (int j = 0; j < m; ++j) {
            double dx = pts[i][0] - pts[j][0], dy = pts[i][1] - pts[j][1], dz = pts[i][2] - pts[j][2];
            if (sqrt(dx * dx + dy * dy + dz * dz) <= 1e-12 * diag) { dup = 1; break; }
        }
        if (!dup) { memcpy(pts[m], pts[i], sizeof(pts[i])); ++m; }
    }
    if (m < 3) return 0.0;
    v3 cen = mk(0, 0, 0);
    for (int i = 0; i < m; ++i) cen = add(cen, mk(pts[i][0], pts[i][1], pts[i][2]));
    cen = scl(cen, 1.0 / m);
    v3 u = fabs(N.x) < 0.9 ? nrm(cross(N, mk(1, 0, 0))) : nrm(cross(N, mk(0, 1, 0)));
    v3 w = cross(N, u);
    for (int i = 0; i < m; ++i) {
        v3 d = sub(mk(pts[i][0], pts[i][1], pts[i][2]), cen);
        pts[i][3] = atan2(dot(d, w), dot(d, u));
    }
    qsort(pts, (size_t)m, sizeof(pts[0]), cmp_angle);
    double a = 0.0;
    for (int i = 0; i < m; ++i) {
        int j = (i + 1) % m;
        v3 d0 = sub(mk(pts[i][0], pts[i][1], pts[i][2]), cen);
        v3 d1 = sub(mk(pts[j][0], pts[j][1], pts[j][2]), cen);
        a += dot(cross(d0, d1), N);
    }
    return 0.5 * fabs(a);
}

/* ------------------------------------------------------------------ */
/* density octree (Sec. 5, Appendix B), sequential                     */
/* ------------------------------------------------------------------ */
#define OCT_FAILED 0x40000000
#define OCT_COUNT_MASK 0x3FFFFFFF
#define OCT_MAX_DEPTH 20
#define OCT_FILL_ITERATIONS 1000
#define OCT_SPLIT_FACTOR 4

typedef struct {
    int32_t* nodes;
    int32_t capacity, alloc, depth, iter, split_count, stop_filling;
    float min_bound[3], size_inv[3], scene_scale, density_scale;
    int64_t block_iter_sum, deposits, rejected, overflow;
} o_octree;

o_octree* orc_octree_create(const float smin[3], const float smax[3], int32_t capacity) {
    if (capacity < 1) return NULL;
    o_octree* o = (o_octree*)calloc(1, sizeof(o_octree));
    float size[3];
    for (int i = 0; i < 3; ++i) {
        size[i] = (smax[i] - smin[i]) * 1.002f;
        o->size_inv[i] = 1.0f / size[i];
    }
    float sq = size[0] * size[0];
    sq = sq + size[1] * size[1];
    sq = sq + size[2] * size[2];
    o->scene_scale = sqrtf(sq);
    const float rel = 0.001f / 1.002f;
    for (int i = 0; i < 3; ++i) o->min_bound[i] = smin[i] - size[i] * rel;
    o->capacity = 1 + ((capacity + 7) & ~7);
    o->nodes = (int32_t*)calloc((size_t)o->capacity, sizeof(int32_t));
    o->alloc = 1;
    o->depth = 0;
    o->iter = 1;
    o->density_scale = 1.0f;
    o->split_count = OCT_SPLIT_FACTOR;
    return o;
}

/* the octree's box as the cell addressing uses it */
void orc_octree_box(const o_octree* o, float min_bound[3], float size_inv[3]) {
    for (int i = 0; i < 3; ++i) {
        min_bound[i] = o->min_bound[i];
        size_inv[i] = o->size_inv[i];
    }
}

void orc_octree_destroy(o_octree* o) {
    if (!o) return;
    free(o->nodes);
    free(o);
}

void orc_octree_set_iteration(o_octree* o, int32_t iter) {
    int32_t ic = iter < OCT_FILL_ITERATIONS ? iter : OCT_FILL_ITERATIONS;
    o->stop_filling = iter > OCT_FILL_ITERATIONS;
    o->density_scale = 1.0f / (float)ic;
    o->split_count = OCT_SPLIT_FACTOR * ic;
    o->iter = iter;
}

void orc_octree_clear_counters(o_octree* o) {
    int32_t n = o->alloc < o->capacity ? o->alloc : o->capacity;
    for (int32_t i = 0; i < n; ++i)
        if (o->nodes[i] > 0) o->nodes[i] = 0;
    /* the ledger restarts: counts are gone, allocated blocks keep existing */
    o->block_iter_sum = 0;
    o->deposits = 0;
}

/* cell addressing in FP32, operation by operation as in Appendix B */
static int norm_pos(const o_octree* o, const float p[3], float np_out[3]) {
    for (int i = 0; i < 3; ++i) {
        float off = p[i] - o->min_bound[i];
        float q = off * o->size_inv[i];
        if (!(q >= 0.0f && q < 1.0f)) return 0;
        np_out[i] = q;
    }
    return 1;
}

static void octree_insert(o_octree* o, const float p[3]) {
    if (o->stop_filling) return;
    float q[3];
    if (!norm_pos(o, p, q)) { o->rejected++; return; }
    int32_t idx = 0, level = 0;
    for (;;) {
        int32_t v = o->nodes[idx];
        if (v < 0) {
            ++level;
            float scale = (float)(1 << level);
            int bx = ((int)(q[0] * scale)) & 1;
            int by = ((int)(q[1] * scale)) & 1;
            int bz = ((int)(q[2] * scale)) & 1;
            idx = -v + bx + 2 * by + 4 * bz;
            continue;
        }
        int32_t cnt = v & OCT_COUNT_MASK;
        o->nodes[idx] = v + 1;
        o->deposits++;
        if (!(v & OCT_FAILED) && level < OCT_MAX_DEPTH && cnt + 1 == o->split_count) {
            int32_t child = o->alloc;
            o->alloc += 8;
            if (child >= o->capacity) {
                o->alloc = o->capacity + 1;
                o->nodes[idx] = (v + 1) | OCT_FAILED;
                o->overflow++;
            } else {
                for (int c = 0; c < 8; ++c) o->nodes[child + c] = o->iter;
                o->nodes[idx] = -child;
                o->block_iter_sum += o->iter;
                if (level + 1 > o->depth) o->depth = level + 1;
            }
        }
        return;
    }
}

void orc_octree_increment(o_octree* o, const float* pos, int64_t n) {
    for (int64_t i = 0; i < n; ++i) octree_insert(o, pos + 3 * i);
}

/* The leaf holding the normalised point q: the word of the leaf and, in
 * *level, its depth.  Below level L the descent takes the child
 * (floor(q * 2^(L+1)) & 1) per axis in FP32, the child the deposits take. */
static int32_t find_leaf(const o_octree* o, const float q[3], int* level) {
    int32_t w = o->nodes[0];
    int L = 0;
    while (w < 0) {
        ++L;
        const float cells = (float)(1 << L);
        int child = 0;
        for (int a = 0; a < 3; ++a) child |= (((int)(q[a] * cells)) & 1) << a;
        w = o->nodes[-w + child];
    }
    *level = L;
    return w;
}

/* Floor under the plane's area in a leaf of diagonal diag, so that a
 * surface grazing a cell does not give an unbounded density (Appendix B):
 * a tenth of diag^2 for the probe at the query point, a hundredth for the
 * offset probes. */
static double area_floor(double diag, int centre) { return diag * diag * (centre ? 0.1 : 0.01); }

/* eq. (octdensity): the count of the leaf holding p over the area of the
 * plane through p (normal n) inside the leaf's box (exact clipping,
 * Appendix A), times the density scale.  centre: the probe at the query
 * point; then *diag_out receives the leaf's diagonal if the leaf has a
 * count.  Cell addressing in FP32, the area in FP64. */
static double leaf_density(const o_octree* o, v3 p, v3 n, int centre, double* diag_out) {
    float pf[3] = {(float)p.x, (float)p.y, (float)p.z}, q[3];
    if (!norm_pos(o, pf, q)) return 0.0;
    int level;
    const int32_t count = find_leaf(o, q, &level) & OCT_COUNT_MASK;
    if (count <= 0) return 0.0;
    const double cells = (double)(1 << level);
    double lo[3], hi[3], rel[3], pp[3] = {p.x, p.y, p.z}, nn[3] = {n.x, n.y, n.z};
    for (int a = 0; a < 3; ++a) {
        const double edge = 1.0 / (cells * (double)o->size_inv[a]);
        lo[a] = (double)(int32_t)(q[a] * (float)(1 << level)) * edge;
        hi[a] = lo[a] + edge;
        rel[a] = pp[a] - (double)o->min_bound[a];
    }
    const double diag = (double)o->scene_scale / cells;
    if (centre && diag_out) *diag_out = diag;
    return (double)o->density_scale * (double)count / fmax(area_floor(diag, centre), orc_exact_area(lo, hi, rel, nn));
}

/* branchless orthonormal basis (Duff et al., JCGT 6(1), 2017) */
static void onb(v3 n, v3* t1, v3* t2) {
    double sgn = copysign(1.0, n.z);
    double a = -1.0 / (sgn + n.z);
    double b = n.x * n.y * a;
    *t1 = mk(1.0 + sgn * n.x * n.x * a, sgn * b, -sgn * n.x);
    *t2 = mk(b, sgn + n.y * n.y * a, -n.y);
}

/* the (k/2)-th smallest of k values (the upper median); sorts v */
static double upper_median(double* v, int k) {
    for (int i = 1; i < k; ++i) {
        const double x = v[i];
        int j = i;
        for (; j > 0 && v[j - 1] > x; --j) v[j] = v[j - 1];
        v[j] = x;
    }
    return v[k / 2];
}

/* Appendix B get_density_robust: eq. (octdensity) at p and at the four
 * points 1.1 leaf diagonals (of p's leaf; 1e-3 scene units when it is
 * empty) away along the tangents; the upper median of the non-zero ones. */
static double octree_density_robust(const o_octree* o, v3 p, v3 n) {
    v3 tx, ty;
    onb(n, &tx, &ty);
    double diag = 1e-3, found[5];
    int k = 0;
    const double centre = leaf_density(o, p, n, 1, &diag);
    if (centre > 0.0) found[k++] = centre;
    const double step = diag * 1.1;
    const v3 away[4] = {add(p, scl(tx, step)), sub(p, scl(tx, step)), add(p, scl(ty, step)), sub(p, scl(ty, step))};
    for (int i = 0; i < 4; ++i) {
        const double r = leaf_density(o, away[i], n, 0, NULL);
        if (r > 0.0) found[k++] = r;
    }
    return k ? upper_median(found, k) : 0.0;
}

double orc_octree_density(o_octree* o, const double p[3], const double n[3], int32_t robust) {
    v3 P = mk(p[0], p[1], p[2]), N = nrm(mk(n[0], n[1], n[2]));
    return robust ? octree_density_robust(o, P, N) : leaf_density(o, P, N, 0, NULL);
}

void orc_octree_density_batch(o_octree* o, const float* pos, const float* nrmv, int64_t n,
                              int32_t robust, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        double q[3] = {nrmv[3 * i], nrmv[3 * i + 1], nrmv[3 * i + 2]};
        out[i] = orc_octree_density(o, p, q, robust);
    }
}

/* info: capacity, allocated (clamped), depth, ledger S, deposits D,
 * overflow events, rejected deposits, sum of block iterations */
int32_t orc_octree_export(const o_octree* o, int32_t* nodes, int32_t cap, int64_t info[8]) {
    int32_t n = o->capacity < cap ? o->capacity : cap;
    if (nodes) memcpy(nodes, o->nodes, sizeof(int32_t) * (size_t)n);
    int64_t leaf_sum = 0;
    int32_t used = o->alloc < o->capacity ? o->alloc : o->capacity;
    for (int32_t i = 0; i < used; ++i)
        if (o->nodes[i] >= 0) leaf_sum += o->nodes[i] & OCT_COUNT_MASK;
    info[0] = o->capacity;
    info[1] = used;
    info[2] = o->depth;
    info[3] = leaf_sum - (int64_t)OCT_SPLIT_FACTOR * o->block_iter_sum;
    info[4] = o->deposits;
    info[5] = o->overflow;
    info[6] = o->rejected;
    info[7] = o->block_iter_sum;
    return n;
}

/* ------------------------------------------------------------------ */
/* scene preprocessing                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t nt, nm, npl, nlights;
    v3 *p0, *p1, *p2, *ng;
    double* area;
    int32_t* mat;
    int32_t* tri_light;            /* light table index of an emissive triangle, else -1 */
    o_material* mats;
    /* light table: emissive triangles first (ascending triangle id), then point lights */
    int32_t* light_tri;            /* triangle id, or -1 for a point light */
    int32_t* light_pl;             /* point light id, or -1 */
    double* light_cdf;
    double* light_psel;
    o_point_light* pl;
    o_camera cam;
    float bmin[3], bmax[3];
    double eps;
} o_scene;

static double emission_weight(const o_material* m) {
    return (m->emission[0] + m->emission[1] + m->emission[2]) / 3.0;
}

o_scene* orc_scene_create(const float* vertices, int32_t nv, const int32_t* tris, const int32_t* tri_mat,
                          int32_t nt, const o_material* mats, int32_t nm, const o_point_light* pl,
                          int32_t npl, const o_camera* cam) {
    if (nt < 1 || nv < 3 || nm < 1) return NULL;
    o_scene* s = (o_scene*)calloc(1, sizeof(o_scene));
    s->nt = nt; s->nm = nm; s->npl = npl;
    s->p0 = malloc(sizeof(v3) * (size_t)nt); s->p1 = malloc(sizeof(v3) * (size_t)nt);
    s->p2 = malloc(sizeof(v3) * (size_t)nt); s->ng = malloc(sizeof(v3) * (size_t)nt);
    s->area = malloc(sizeof(double) * (size_t)nt);
    s->mat = malloc(sizeof(int32_t) * (size_t)nt);
    s->tri_light = malloc(sizeof(int32_t) * (size_t)nt);
    s->mats = malloc(sizeof(o_material) * (size_t)nm);
    memcpy(s->mats, mats, sizeof(o_material) * (size_t)nm);
    s->pl = malloc(sizeof(o_point_light) * (size_t)(npl > 0 ? npl : 1));
    if (npl > 0) memcpy(s->pl, pl, sizeof(o_point_light) * (size_t)npl);
    s->cam = *cam;
    for (int i = 0; i < 3; ++i) { s->bmin[i] = vertices[i]; s->bmax[i] = vertices[i]; }
    for (int32_t v = 0; v < nv; ++v)
        for (int i = 0; i < 3; ++i) {
            float x = vertices[3 * v + i];
            if (x < s->bmin[i]) s->bmin[i] = x;
            if (x > s->bmax[i]) s->bmax[i] = x;
        }
    s->eps = 1e-5 * len(sub(from_f(s->bmax), from_f(s->bmin)));
    int32_t ne = 0;
    for (int32_t t = 0; t < nt; ++t) {
        s->p0[t] = from_f(vertices + 3 * tris[3 * t]);
        s->p1[t] = from_f(vertices + 3 * tris[3 * t + 1]);
        s->p2[t] = from_f(vertices + 3 * tris[3 * t + 2]);
        v3 c = cross(sub(s->p1[t], s->p0[t]), sub(s->p2[t], s->p0[t]));
        double l = len(c);
        s->area[t] = 0.5 * l;
        s->ng[t] = l > 0 ? scl(c, 1.0 / l) : mk(0, 0, 1);
        s->mat[t] = tri_mat[t];
        s->tri_light[t] = -1;
        if (emission_weight(&mats[tri_mat[t]]) > 0.0 && l > 0) ++ne;
    }
    s->nlights = ne + npl;
    int32_t nl = s->nlights > 0 ? s->nlights : 1;
    s->light_tri = malloc(sizeof(int32_t) * (size_t)nl);
    s->light_pl = malloc(sizeof(int32_t) * (size_t)nl);
    s->light_cdf = malloc(sizeof(double) * (size_t)nl);
    s->light_psel = malloc(sizeof(double) * (size_t)nl);
    double* w = malloc(sizeof(double) * (size_t)nl);
    int32_t k = 0;
    for (int32_t t = 0; t < nt; ++t)
        if (emission_weight(&mats[tri_mat[t]]) > 0.0 && s->area[t] > 0) {
            s->light_tri[k] = t; s->light_pl[k] = -1;
            s->tri_light[t] = k;
            w[k] = PI * s->area[t] * emission_weight(&mats[tri_mat[t]]);
            ++k;
        }
    for (int32_t i = 0; i < npl; ++i) {
        s->light_tri[k] = -1; s->light_pl[k] = i;
        w[k] = (pl[i].power[0] + pl[i].power[1] + pl[i].power[2]) / 3.0;
        ++k;
    }
    double tot = 0.0;
    for (int32_t i = 0; i < s->nlights; ++i) tot += w[i];
    double acc = 0.0;
    for (int32_t i = 0; i < s->nlights; ++i) {
        acc += w[i];
        s->light_cdf[i] = acc / tot;
        s->light_psel[i] = w[i] / tot;
    }
    if (s->nlights > 0) s->light_cdf[s->nlights - 1] = 1.0;
    free(w);
    return s;
}

void orc_scene_destroy(o_scene* s) {
    if (!s) return;
    free(s->p0); free(s->p1); free(s->p2); free(s->ng); free(s->area); free(s->mat);
    free(s->tri_light); free(s->mats); free(s->pl); free(s->light_tri); free(s->light_pl);
    free(s->light_cdf); free(s->light_psel);
    free(s);
}

void orc_scene_bounds(const o_scene* s, float bmin[3], float bmax[3]) {
    memcpy(bmin, s->bmin, sizeof(float) * 3);
    memcpy(bmax, s->bmax, sizeof(float) * 3);
}

/* ------------------------------------------------------------------ */
/* ray casting: brute force over all triangles                         */
/* ------------------------------------------------------------------ */
/* Moeller-Trumbore in FP64; closest t > 0, ties go to the lowest id */
static int closest_hit(const o_scene* s, v3 o, v3 d, double* t_out) {
    double best = INFINITY;
    int prim = -1;
    for (int32_t t = 0; t < s->nt; ++t) {
        v3 e1 = sub(s->p1[t], s->p0[t]), e2 = sub(s->p2[t], s->p0[t]);
        v3 pv = cross(d, e2);
        double det = dot(e1, pv);
        if (det == 0.0) continue;
        double inv = 1.0 / det;
        v3 tv = sub(o, s->p0[t]);
        double u = dot(tv, pv) * inv;
        if (u < 0.0 || u > 1.0) continue;
        v3 qv = cross(tv, e1);
        double v = dot(d, qv) * inv;
        if (v < 0.0 || u + v > 1.0) continue;
        double tt = dot(e2, qv) * inv;
        if (tt > 0.0 && tt < best) { best = tt; prim = t; }
    }
    *t_out = best;
    return prim;
}

static int occluded(const o_scene* s, v3 o, v3 d, double tmax) {
    for (int32_t t = 0; t < s->nt; ++t) {
        v3 e1 = sub(s->p1[t], s->p0[t]), e2 = sub(s->p2[t], s->p0[t]);
        v3 pv = cross(d, e2);
        double det = dot(e1, pv);
        if (det == 0.0) continue;
        double inv = 1.0 / det;
        v3 tv = sub(o, s->p0[t]);
        double u = dot(tv, pv) * inv;
        if (u < 0.0 || u > 1.0) continue;
        v3 qv = cross(tv, e1);
        double v = dot(d, qv) * inv;
        if (v < 0.0 || u + v > 1.0) continue;
        double tt = dot(e2, qv) * inv;
        if (tt > 0.0 && tt < tmax) return 1;
    }
    return 0;
}

int32_t orc_closest_hit(const o_scene* s, const double o[3], const double d[3], double* t) {
    return closest_hit(s, mk(o[0], o[1], o[2]), mk(d[0], d[1], d[2]), t);
}

static v3 offset_origin(const o_scene* s, v3 x, v3 n, v3 dir) {
    return dot(dir, n) > 0.0 ? add(x, scl(n, s->eps)) : sub(x, scl(n, s->eps));
}

/* ------------------------------------------------------------------ */
/* BSDFs (geometric normal only).  Directions point away from the       */
/* surface; wi is where the path came from, wo where it goes.           */
/* ------------------------------------------------------------------ */
static int mat_is_delta(const o_material* m) { return m->type == M_MIRROR || m->type == M_DIELECTRIC; }
static int mat_is_black(const o_material* m) {
    return m->albedo[0] == 0.0f && m->albedo[1] == 0.0f && m->albedo[2] == 0.0f;
}
static v3 albedo(const o_material* m) { return from_f(m->albedo); }

static double fresnel_dielectric(double cos_i, double eta) {
    /* eta = n_incident / n_transmitted; cos_i >= 0 */
    double sin2t = eta * eta * (1.0 - cos_i * cos_i);
    if (sin2t >= 1.0) return 1.0;
    double cos_t = sqrt(1.0 - sin2t);
    double rs = (eta * cos_i - cos_t) / (eta * cos_i + cos_t);
    double rp = (cos_i - eta * cos_t) / (cos_i + eta * cos_t);
    return 0.5 * (rs * rs + rp * rp);
}

static double dielectric_F(const o_material* m, v3 n, v3 wi) {
    double c = dot(wi, n);
    double eta = c > 0.0 ? 1.0 / (double)m->ior : (double)m->ior;
    return fresnel_dielectric(fabs(c), eta);
}

/* GGX (Walter et al., EGSR 2007) */
static double ggx_D(double alpha, double cos_m) {
    if (cos_m <= 0.0) return 0.0;
    double a2 = alpha * alpha;
    double t = cos_m * cos_m * (a2 - 1.0) + 1.0;
    return a2 / (PI * t * t);
}
static double ggx_G1(double alpha, double cos_v) {
    double c2 = cos_v * cos_v;
    double tan2 = (1.0 - c2) / c2;
    return 2.0 / (1.0 + sqrt(1.0 + alpha * alpha * tan2));
}

/* f(wi, wo) */
static v3 bsdf_f(const o_material* m, v3 n, v3 wi, v3 wo) {
    double ci = dot(n, wi), co = dot(n, wo);
    if (ci * co <= 0.0) return mk(0, 0, 0);
    if (m->type == M_LAMBERT) return scl(albedo(m), 1.0 / PI);
    if (m->type == M_GGX) {
        v3 ns = ci > 0 ? n : scl(n, -1.0);
        v3 h = nrm(add(wi, wo));
        double a = m->alpha;
        double D = ggx_D(a, dot(h, ns));
        double G = ggx_G1(a, fabs(ci)) * ggx_G1(a, fabs(co));
        return scl(albedo(m), D * G / (4.0 * fabs(ci) * fabs(co)));
    }
    return mk(0, 0, 0);     /* delta lobes have no finite value */
}

/* solid-angle pdf of sampling wo given wi (discrete probability for delta lobes) */
static double bsdf_pdf(const o_material* m, v3 n, v3 wi, v3 wo) {
    double ci = dot(n, wi), co = dot(n, wo);
    int same = ci * co > 0.0;
    switch (m->type) {
    case M_LAMBERT: return same ? fabs(co) / PI : 0.0;
    case M_MIRROR: return same ? 1.0 : 0.0;
    case M_DIELECTRIC: {
        double F = dielectric_F(m, n, wi);
        return same ? F : 1.0 - F;
    }
    case M_GGX: {
        if (!same) return 0.0;
        v3 ns = ci > 0 ? n : scl(n, -1.0);
        v3 h = nrm(add(wi, wo));
        double cm = dot(h, ns);
        return ggx_D(m->alpha, cm) * cm / (4.0 * fabs(dot(wo, h)));
    }
    }
    return 0.0;
}

typedef struct { v3 dir; v3 weight; double pdf; int event; int ok; } bsdf_sample;

static bsdf_sample sample_bsdf(const o_material* m, v3 n, v3 wi, const double u[4]) {
    bsdf_sample r;
    memset(&r, 0, sizeof(r));
    double ci = dot(n, wi);
    if (ci == 0.0) return r;
    v3 ns = ci > 0 ? n : scl(n, -1.0);
    switch (m->type) {
    case M_LAMBERT: {
        v3 t1, t2;
        onb(ns, &t1, &t2);
        double rr = sqrt(u[1]), phi = 2.0 * PI * u[2];
        double z = sqrt(fmax(0.0, 1.0 - u[1]));
        r.dir = nrm(add(add(scl(t1, rr * cos(phi)), scl(t2, rr * sin(phi))), scl(ns, z)));
        double co = dot(r.dir, ns);
        if (co <= 0.0) return r;
        r.pdf = co / PI;
        r.weight = albedo(m);
        r.event = EV_SCATTER;
        r.ok = 1;
        return r;
    }
    case M_MIRROR: {
        double c = dot(wi, ns);
        r.dir = sub(scl(ns, 2.0 * c), wi);
        r.pdf = 1.0;
        r.weight = albedo(m);
        r.event = EV_REFLECT;
        r.ok = 1;
        return r;
    }
    case M_DIELECTRIC: {
        double c = dot(wi, ns);
        double eta = ci > 0.0 ? 1.0 / (double)m->ior : (double)m->ior;
        double F = fresnel_dielectric(c, eta);
        if (u[0] < F) {
            r.dir = sub(scl(ns, 2.0 * c), wi);
            r.pdf = F;
            r.event = EV_REFLECT;
        } else {
            double sin2t = eta * eta * (1.0 - c * c);
            double ct = sqrt(fmax(0.0, 1.0 - sin2t));
            r.dir = nrm(sub(scl(ns, eta * c - ct), scl(wi, eta)));
            r.pdf = 1.0 - F;
            r.event = EV_REFRACT;
        }
        r.weight = albedo(m);
        r.ok = 1;
        return r;
    }
    case M_GGX: {
        double a = m->alpha;
        double tan_t = a * sqrt(u[1] / (1.0 - u[1]));
        double cos_t = 1.0 / sqrt(1.0 + tan_t * tan_t);
        double sin_t = tan_t * cos_t;
        double phi = 2.0 * PI * u[2];
        v3 t1, t2;
        onb(ns, &t1, &t2);
        v3 h = nrm(add(add(scl(t1, sin_t * cos(phi)), scl(t2, sin_t * sin(phi))), scl(ns, cos_t)));
        double wh = dot(wi, h);
        if (wh <= 0.0) return r;
        r.dir = sub(scl(h, 2.0 * wh), wi);
        double co = dot(r.dir, ns);
        if (co <= 0.0) return r;
        double cim = fabs(ci);
        double G = ggx_G1(a, cim) * ggx_G1(a, co);
        r.pdf = ggx_D(a, cos_t) * cos_t / (4.0 * wh);
        r.weight = scl(albedo(m), G * wh / (cim * cos_t));
        r.event = EV_SCATTER;
        r.ok = 1;
        return r;
    }
    }
    return r;
}

/* exported for the oracle's own unit tests */
void orc_bsdf_eval(const o_material* m, const double n[3], const double wi[3], const double wo[3],
                   double f[3], double* pdf) {
    v3 N = mk(n[0], n[1], n[2]), I = mk(wi[0], wi[1], wi[2]), O = mk(wo[0], wo[1], wo[2]);
    v3 r = bsdf_f(m, N, I, O);
    f[0] = r.x; f[1] = r.y; f[2] = r.z;
    *pdf = bsdf_pdf(m, N, I, O);
}

int32_t orc_bsdf_sample(const o_material* m, const double n[3], const double wi[3], const double u[3],
                        double dir[3], double weight[3], double* pdf) {
    double uu[4] = {u[0], u[1], u[2], 0.0};
    bsdf_sample s = sample_bsdf(m, mk(n[0], n[1], n[2]), mk(wi[0], wi[1], wi[2]), uu);
    dir[0] = s.dir.x; dir[1] = s.dir.y; dir[2] = s.dir.z;
    weight[0] = s.weight.x; weight[1] = s.weight.y; weight[2] = s.weight.z;
    *pdf = s.pdf;
    return s.ok ? s.event : 0;
}

/* ------------------------------------------------------------------ */
/* camera                                                              */
/* ------------------------------------------------------------------ */
typedef struct { v3 eye, f, r, u; double tan_half, aspect; int w, h; } o_cam;

static o_cam make_cam(const o_camera* c, int w, int h) {
    o_cam k;
    k.eye = from_f(c->eye);
    k.f = nrm(sub(from_f(c->look_at), k.eye));
    k.r = nrm(cross(k.f, from_f(c->up)));
    k.u = cross(k.r, k.f);
    k.tan_half = tan(0.5 * (double)c->vfov_deg * PI / 180.0);
    k.aspect = (double)w / (double)h;
    k.w = w; k.h = h;
    return k;
}

static v3 cam_dir(const o_cam* k, int px, int py, double u0, double u1) {
    double sx = (2.0 * ((double)px + u0) / k->w - 1.0) * k->tan_half * k->aspect;
    double sy = (1.0 - 2.0 * ((double)py + u1) / k->h) * k->tan_half;
    return nrm(add(k->f, add(scl(k->r, sx), scl(k->u, sy))));
}

/* density of primary hits per unit area per iteration (test hook) */
static double camera_hit_density(const o_cam* k, v3 x, v3 n) {
    v3 d = sub(x, k->eye);
    double dist2 = dot(d, d);
    v3 w = scl(d, 1.0 / sqrt(dist2));
    double c = dot(w, k->f);
    if (c <= 0.0) return 0.0;
    double sx = dot(w, k->r) / c, sy = dot(w, k->u) / c;
    if (fabs(sx) > k->tan_half * k->aspect || fabs(sy) > k->tan_half) return 0.0;
    double film = 4.0 * k->tan_half * k->tan_half * k->aspect;
    double pdf_w = 1.0 / (film * c * c * c);
    return (double)k->w * (double)k->h * pdf_w * fabs(dot(n, w)) / dist2;
}

/* ------------------------------------------------------------------ */
/* explicit MIS over a whole path                                       */
/* ------------------------------------------------------------------ */
/* A path of length L (segments) with vertices x_0 (camera) .. x_L (light).
 * Segment i joins x_i and x_{i+1}; its endpoints are given separately
 * (seg_a[i] at x_i, seg_b[i] at x_{i+1}) together with the normals used
 * for the area conversion at each end, so that a merged path can take the
 * photon hit's geometry for the photon segment.  Vertices 1..L-1 carry a
 * material and a shading normal for BSDF pdfs. */
#define MAXL 64
typedef struct {
    int L;
    v3 seg_a[MAXL], seg_b[MAXL], na[MAXL], nb[MAXL];
    const o_material* mat[MAXL];
    v3 vn[MAXL];
    double p_light;        /* light sampling density (area measure; selection prob for point lights) */
    int hittable;          /* area light: can be found by a random hit */
    double rho;            /* density of NEE vertices at x_{L-1} */
    double r2pi;           /* pi r^2 */
    int photons;           /* n_P > 0 */
    double n_lp;           /* n_LP, light photons per iteration (0 = none) */
    double n_e;            /* n_E, NEE samples at x_{L-1} (1; with NEE recycling the events found there) */
} o_path;

/* index of the conventional-photon technique LP_k in the technique list */
static int lp_tech(int L, int k) { return 1 + (L >= 2 ? L - 2 : 0) + k; }
static int n_techniques(int L) { return 2 + (L >= 2 ? L - 2 : 0) + (L >= 1 ? L - 1 : 0); }

/* returns all technique densities: out[0] = e, out[1] = E, out[1+k] = P_k
 * (k = 1 .. L-2), out[lp_tech(L, k)] = LP_k (k = 1 .. L-1) */
static void path_densities(const o_path* P, double* out) {
    int L = P->L;
    double f[MAXL], r[MAXL];
    for (int i = 1; i <= L - 1; ++i) {
        v3 wprev = nrm(sub(P->seg_a[i - 1], P->seg_b[i - 1]));
        v3 d = sub(P->seg_b[i], P->seg_a[i]);
        double d2 = dot(d, d);
        v3 wnext = scl(d, 1.0 / sqrt(d2));
        f[i] = bsdf_pdf(P->mat[i], P->vn[i], wprev, wnext) * fabs(dot(P->nb[i], wnext)) / d2;
    }
    for (int i = 1; i <= L - 2; ++i) {
        /* p_{i+1 -> i}: BSDF at x_{i+1} given the direction to x_{i+2} */
        v3 d = sub(P->seg_a[i], P->seg_b[i]);
        double d2 = dot(d, d);
        v3 wback = scl(d, 1.0 / sqrt(d2));
        v3 wfwd = nrm(sub(P->seg_b[i + 1], P->seg_a[i + 1]));
        r[i] = bsdf_pdf(P->mat[i + 1], P->vn[i + 1], wfwd, wback) * fabs(dot(P->na[i], wback)) / d2;
    }
    double pe = 0.0;
    if (P->hittable) {
        pe = 1.0;
        for (int i = 1; i <= L - 1; ++i) pe *= f[i];
    }
    out[0] = pe;
    double pE = 0.0;
    if (L >= 2 && !mat_is_delta(P->mat[L - 1])) {
        pE = P->p_light;
        for (int i = 1; i <= L - 2; ++i) pE *= f[i];
    }
    out[1] = P->n_e * pE;
    for (int k = 1; k <= L - 2; ++k) {
        double pp = 0.0;
        if (P->photons && P->rho > 0.0 && !mat_is_delta(P->mat[k])) {
            pp = P->p_light * P->rho * P->r2pi;
            for (int i = k; i <= L - 2; ++i) pp *= r[i];
            for (int i = 1; i <= k - 1; ++i) pp *= f[i];
        }
        out[1 + k] = pp;
    }
    /* conventional light photons, eq. (stdphotonpdf): the light point (p_light),
     * the emission toward x_{L-1} (p_{L -> L-1}: cosine lobe of an area light,
     * uniform sphere of a point light, converted to area at x_{L-1}), the
     * backward walk down to x_k, the camera walk up to x_k and the merge
     * disc pi r^2; n_LP photons per iteration */
    double rl = 0.0;
    if (L >= 1) {
        v3 d = sub(P->seg_b[L - 1], P->seg_a[L - 1]);
        double d2 = dot(d, d);
        v3 w = scl(d, 1.0 / sqrt(d2));
        double emit = P->hittable ? fmax(0.0, -dot(P->nb[L - 1], w)) / PI : 1.0 / (4.0 * PI);
        rl = emit * fabs(dot(P->na[L - 1], w)) / d2;
    }
    for (int k = 1; k <= L - 1; ++k) {
        double q = 0.0;
        if (P->n_lp > 0.0 && !mat_is_delta(P->mat[k])) {
            q = P->n_lp * P->p_light * P->r2pi * rl;
            for (int i = k; i <= L - 2; ++i) q *= r[i];
            for (int i = 1; i <= k - 1; ++i) q *= f[i];
        }
        out[lp_tech(L, k)] = q;
    }
}

/* tech: 0 = e, 1 = E, 1 + k = P_k, lp_tech(L, k) = LP_k */
static double mis_weight(const o_path* P, int tech) {
    double pd[2 * MAXL + 2];
    path_densities(P, pd);
    int nt = n_techniques(P->L);
    double sum = 0.0;
    for (int i = 0; i < nt; ++i) sum += pd[i];
    if (!(sum > 0.0)) return 0.0;
    return pd[tech] / sum;
}

/* ------------------------------------------------------------------ */
/* render                                                              */
/* ------------------------------------------------------------------ */
typedef struct {
    int nhit;                     /* number of hits (vertices 1..nhit) */
} path_hdr;

typedef struct { int tri, pl; v3 x, n; double p_light, d2, dist; v3 w, dE; int hittable; } light_sample;

typedef struct {
    const o_scene* s;
    const o_params* prm;
    o_cam cam;
    rng_key key;
    int npath, L, win_w;
    /* per path, per depth 0..L */
    v3 *pos, *nrml, *wo, *tau;
    int *mat, *prim, *vid, *nhit, *pixel;
    /* vertices in canonical order */
    int nvert;
    int *v_path, *v_depth;
    double* v_rho;
    double* v_pos;                /* positions of this iteration's vertices, 3 per vertex */
    double* v_ne;                 /* n_E per vertex: 1, or with NEE recycling the NEE vertices within the radius */
    light_sample* v_ls;           /* each vertex's own light sample (NEE recycling) */
    int* v_lsok;                  /* 1 when that sample is unoccluded with nonzero dE */
    /* emission events */
    int nev, cap_ev;
    int *ev_path, *ev_depth, *ev_tri;
    v3* ev_val;
    o_octree* oct;
} o_iter;

#define IDX(it, p, k) ((size_t)(p) * (size_t)((it)->L + 1) + (size_t)(k))

static void trace_camera_path(o_iter* it, int p, int iter, o_record* rec) {
    const o_scene* s = it->s;
    int pix = it->pixel[p];
    int px = pix % it->prm->width, py = pix / it->prm->width;
    double u[4];
    uniforms(it->key, (uint32_t)pix, (uint32_t)iter, 0u, TAG_CAMERA, u);
    v3 o = it->cam.eye, d = cam_dir(&it->cam, px, py, u[0], u[1]);
    v3 tau = mk(1, 1, 1);
    it->pos[IDX(it, p, 0)] = o;
    int nh = 0;
    for (int k = 1; k <= it->L; ++k) {
        double t;
        int prim = closest_hit(s, o, d, &t);
        o_record* rc = rec ? &rec[(size_t)p * (size_t)it->L + (size_t)(k - 1)] : NULL;
        if (prim < 0) {
            if (rc) { rc->type = EV_ESCAPE; rc->mat = -1; rc->prim = -1; }
            break;
        }
        v3 x = add(o, scl(d, t));
        v3 n = s->ng[prim];
        const o_material* m = &s->mats[s->mat[prim]];
        v3 wo = scl(d, -1.0);
        size_t id = IDX(it, p, k);
        it->pos[id] = x; it->nrml[id] = n; it->wo[id] = wo; it->tau[id] = tau;
        it->mat[id] = s->mat[prim]; it->prim[id] = prim;
        nh = k;
        if (rc) {
            rc->mat = s->mat[prim]; rc->prim = prim;
            rc->pos[0] = (float)x.x; rc->pos[1] = (float)x.y; rc->pos[2] = (float)x.z;
            rc->type = EV_STOP;
        }
        if (emission_weight(m) > 0.0 && dot(n, wo) > 0.0 && s->tri_light[prim] >= 0) {
#ifdef _OPENMP
#pragma omp critical(ev)
#endif
            {
                if (it->nev == it->cap_ev) {
                    it->cap_ev = it->cap_ev * 2 + 64;
                    it->ev_path = realloc(it->ev_path, sizeof(int) * (size_t)it->cap_ev);
                    it->ev_depth = realloc(it->ev_depth, sizeof(int) * (size_t)it->cap_ev);
                    it->ev_tri = realloc(it->ev_tri, sizeof(int) * (size_t)it->cap_ev);
                    it->ev_val = realloc(it->ev_val, sizeof(v3) * (size_t)it->cap_ev);
                }
                it->ev_path[it->nev] = p; it->ev_depth[it->nev] = k; it->ev_tri[it->nev] = prim;
                it->ev_val[it->nev] = hmul(tau, from_f(m->emission));
                it->nev++;
            }
        }
        if (mat_is_black(m) || k == it->L) break;
        it->vid[id] = 1;          /* marks a stored NEE vertex; numbered later */
        uniforms(it->key, (uint32_t)pix, (uint32_t)iter, (uint32_t)k, TAG_BSDF, u);
        bsdf_sample bs = sample_bsdf(m, n, wo, u);
        if (!bs.ok) break;
        if (rc) rc->type = bs.event;
        tau = hmul(tau, bs.weight);
        o = offset_origin(s, x, n, bs.dir);
        d = bs.dir;
    }
    it->nhit[p] = nh;
}

/* fill the segments of camera path p up to depth k (x_0 .. x_k) */
static void path_from_camera(const o_iter* it, int p, int k, o_path* P) {
    for (int i = 0; i < k; ++i) {
        P->seg_a[i] = it->pos[IDX(it, p, i)];
        P->seg_b[i] = it->pos[IDX(it, p, i + 1)];
        P->na[i] = i > 0 ? it->nrml[IDX(it, p, i)] : it->cam.f;
        P->nb[i] = it->nrml[IDX(it, p, i + 1)];
    }
    for (int i = 1; i <= k; ++i) {
        P->mat[i] = &it->s->mats[it->mat[IDX(it, p, i)]];
        P->vn[i] = it->nrml[IDX(it, p, i)];
    }
}

static light_sample sample_light(const o_iter* it, v3 x, v3 nx, const double u[4]) {
    const o_scene* s = it->s;
    light_sample ls;
    memset(&ls, 0, sizeof(ls));
    ls.tri = -1; ls.pl = -1;
    if (s->nlights == 0) return ls;
    int li = 0;
    while (li < s->nlights - 1 && !(u[0] < s->light_cdf[li])) ++li;
    double psel = s->light_psel[li];
    if (s->light_tri[li] >= 0) {
        int t = s->light_tri[li];
        double su = sqrt(u[1]);
        double b0 = 1.0 - su, b1 = u[2] * su;
        v3 y = add(add(scl(s->p0[t], b0), scl(s->p1[t], b1)), scl(s->p2[t], 1.0 - b0 - b1));
        v3 dv = sub(y, x);
        double d2 = dot(dv, dv), dist = sqrt(d2);
        v3 w = scl(dv, 1.0 / dist);
        ls.tri = t; ls.x = y; ls.n = s->ng[t]; ls.d2 = d2; ls.dist = dist; ls.w = w;
        ls.p_light = psel / s->area[t];
        ls.hittable = 1;
        double cl = -dot(ls.n, w), cx = fabs(dot(nx, w));
        if (cl > 0.0 && cx > 0.0)
            ls.dE = scl(from_f(s->mats[s->mat[t]].emission), cx * cl / (d2 * ls.p_light));
    } else {
        const o_point_light* l = &s->pl[s->light_pl[li]];
        v3 y = from_f(l->pos);
        v3 dv = sub(y, x);
        double d2 = dot(dv, dv), dist = sqrt(d2);
        v3 w = scl(dv, 1.0 / dist);
        ls.pl = s->light_pl[li]; ls.x = y; ls.n = scl(w, -1.0); ls.d2 = d2; ls.dist = dist; ls.w = w;
        ls.p_light = psel;
        ls.hittable = 0;
        double cx = fabs(dot(nx, w));
        if (cx > 0.0) ls.dE = scl(from_f(l->power), cx / (4.0 * PI * d2 * psel));
    }
    return ls;
}

/* The two density estimators Sec. 5 compares the octree with, over this
 * iteration's NEE vertices only (3-D distances, per unit area per
 * iteration):
 *  - mode 4, fixed radius (the naive estimator): the number of vertices
 *    within R of x, over pi R^2;
 *  - mode 5, k nearest neighbours: k / (pi d_k^2), d_k the distance from x
 *    to its k-th nearest vertex (a vertex at x is its own nearest); when
 *    fewer than k vertices lie within R, the mode-4 estimate. */
static double set_density(const double* pts, int n, v3 x, int mode, double R, int k) {
    double R2 = R * R, best[64];
    int m = 0;
    for (int i = 0; i < n; ++i) {
        v3 d = sub(mk(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]), x);
        double d2 = dot(d, d);
        if (!(d2 < R2)) continue;
        if (mode == 5) {
            /* keep the k smallest squared distances, ascending */
            int j = m < k ? m : k - 1;
            if (m >= k && d2 >= best[k - 1]) { ++m; continue; }
            while (j > 0 && best[j - 1] > d2) { best[j] = best[j - 1]; --j; }
            best[j] = d2;
        }
        ++m;
    }
    if (mode == 5 && m >= k) return (double)k / (PI * best[k - 1]);
    return (double)m / (PI * R2);
}

static double query_density(const o_iter* it, v3 x, v3 n) {
    const o_params* p = it->prm;
    switch (p->density_mode) {
    case 0: return leaf_density(it->oct, x, n, 0, NULL);
    case 1: return octree_density_robust(it->oct, x, n);
    case 3: return p->analytic_rho0 + p->analytic_cam_weight * camera_hit_density(&it->cam, x, n);
    case 4:
    case 5: return set_density(it->v_pos, it->nvert, x, p->density_mode, p->density_radius, p->knn_k);
    }
    return 0.0;
}

/* test hook: the mode-4/5 estimators of n_query points over a point set */
int32_t orc_point_density(const double* pts, int32_t n, const double* q, int32_t n_query, int32_t mode,
                          double radius, int32_t k, double* out) {
    if (n < 0 || n_query < 0 || (mode != 4 && mode != 5) || !(radius > 0.0) || k < 1 || k > 64) return -1;
    for (int32_t i = 0; i < n_query; ++i)
        out[i] = set_density(pts, n, mk(q[3 * i], q[3 * i + 1], q[3 * i + 2]), mode, radius, k);
    return 0;
}

typedef struct { double *e, *E, *P, *LP; o_stats st; } o_accum;

static void add_px(double* img, int pix, v3 c) {
    img[3 * pix] += c.x; img[3 * pix + 1] += c.y; img[3 * pix + 2] += c.z;
}

/* pass 2 for one NEE vertex: NEE contribution, then the photon walk */
static void nee_and_photon(const o_iter* it, int vi, int iter, o_accum* acc) {
    const o_scene* s = it->s;
    const o_params* prm = it->prm;
    int p = it->v_path[vi], m = it->v_depth[vi];
    size_t id = IDX(it, p, m);
    v3 x = it->pos[id], n = it->nrml[id], wo = it->wo[id], tau = it->tau[id];
    const o_material* mt = &s->mats[it->mat[id]];
    int pix = it->pixel[p];
    double rho = it->v_rho[vi];
    double u[4];
    uniforms(it->key, (uint32_t)pix, (uint32_t)iter, (uint32_t)m, TAG_NEE, u);
    light_sample ls = sample_light(it, x, n, u);
    const int recycle = prm->nee_radius > 0.0;
    if (recycle) { it->v_ls[vi] = ls; it->v_lsok[vi] = 0; }
    if (is_zero(ls.dE)) return;
    v3 so = offset_origin(s, x, n, ls.w);
    v3 sd = sub(ls.x, so);
    double sl = len(sd);
    acc->st.rays += 1;
    if (occluded(s, so, scl(sd, 1.0 / sl), (1.0 - 1e-5) * sl)) return;
    acc->st.nee_visible += 1;
    if (recycle) it->v_lsok[vi] = 1;
    double r2pi = PI * prm->merge_radius * prm->merge_radius;
    if (!recycle && !mat_is_delta(mt)) {
        v3 f = bsdf_f(mt, n, wo, ls.w);
        if (!is_zero(f)) {
            o_path P;
            P.L = m + 1;
            path_from_camera(it, p, m, &P);
            P.seg_a[m] = x; P.seg_b[m] = ls.x; P.na[m] = n; P.nb[m] = ls.n;
            P.p_light = ls.p_light; P.hittable = ls.hittable; P.rho = rho; P.r2pi = r2pi;
            P.photons = prm->enable_photons;
            P.n_lp = prm->light_photons;
            P.n_e = 1.0;
            double w = mis_weight(&P, 1);
            add_px(acc->E, pix, scl(hmul(hmul(tau, f), ls.dE), w));
        }
    }
    if (!prm->enable_photons || !(rho > 0.0)) return;
    /* photon from this virtual light: flux dE / rho, first scatter at x with
     * the NEE direction as incident direction */
    v3 phi = scl(ls.dE, 1.0 / rho);
    acc->st.photons += 1;
    int L = prm->max_path_len;
    v3 ypos[MAXL], yn[MAXL];
    const o_material* ymat[MAXL];
    ypos[0] = x; yn[0] = n; ymat[0] = mt;
    uniforms(it->key, (uint32_t)pix, (uint32_t)iter, (uint32_t)(16 * m), TAG_PHOTON, u);
    bsdf_sample bs = sample_bsdf(mt, n, ls.w, u);
    if (!bs.ok) return;
    phi = hmul(phi, bs.weight);
    v3 o = offset_origin(s, x, n, bs.dir), d = bs.dir;
    for (int j = 1; j <= L - 2; ++j) {
        double t;
        int prim = closest_hit(s, o, d, &t);
        acc->st.rays += 1;
        if (prim < 0) break;
        acc->st.photon_segments += 1;
        v3 y = add(o, scl(d, t));
        v3 ny = s->ng[prim];
        const o_material* my = &s->mats[s->mat[prim]];
        ypos[j] = y; yn[j] = ny; ymat[j] = my;
        if (!mat_is_delta(my)) {
            double r = prm->merge_radius;
            v3 wd = scl(d, -1.0);
            for (int q = 0; q < it->nvert; ++q) {
                int k = it->v_depth[q];
                if (k + j + 1 > L) continue;
                size_t qid = IDX(it, it->v_path[q], k);
                v3 dq = sub(it->pos[qid], y);
                if (dot(dq, dq) >= r * r) continue;
                const o_material* mq = &s->mats[it->mat[qid]];
                if (mat_is_delta(mq)) continue;
                v3 f = bsdf_f(mq, it->nrml[qid], it->wo[qid], wd);
                if (is_zero(f)) continue;
                o_path P;
                P.L = k + j + 1;
                path_from_camera(it, it->v_path[q], k, &P);
                /* photon segment: from the merge point (photon hit geometry) back to y_{j-1} */
                P.seg_a[k] = y; P.seg_b[k] = ypos[j - 1]; P.na[k] = ny; P.nb[k] = yn[j - 1];
                for (int i = 1; i <= j - 1; ++i) {
                    P.seg_a[k + i] = ypos[j - i]; P.seg_b[k + i] = ypos[j - i - 1];
                    P.na[k + i] = yn[j - i]; P.nb[k + i] = yn[j - i - 1];
                    P.mat[k + i] = ymat[j - i]; P.vn[k + i] = yn[j - i];
                }
                P.mat[k + j] = ymat[0]; P.vn[k + j] = yn[0];
                P.seg_a[k + j] = ypos[0]; P.seg_b[k + j] = ls.x; P.na[k + j] = yn[0]; P.nb[k + j] = ls.n;
                P.p_light = ls.p_light; P.hittable = ls.hittable; P.rho = rho; P.r2pi = r2pi;
                P.photons = 1;
                P.n_lp = prm->light_photons;
                P.n_e = it->v_ne[vi];
                double w = mis_weight(&P, 1 + k);
                v3 c = scl(hmul(hmul(it->tau[qid], f), phi), w / r2pi);
                add_px(acc->P, it->pixel[it->v_path[q]], c);
                acc->st.merges += 1;
            }
        }
        if (j == L - 2 || mat_is_black(my)) break;
        uniforms(it->key, (uint32_t)pix, (uint32_t)iter, (uint32_t)(16 * m + j), TAG_PHOTON, u);
        bs = sample_bsdf(my, ny, scl(d, -1.0), u);
        if (!bs.ok) break;
        phi = hmul(phi, bs.weight);
        o = offset_origin(s, y, ny, bs.dir);
        d = bs.dir;
    }
}

/* NEE recycling (Sec. 6, the subsection on reusing NEE events): vertex vi
 * evaluates the light samples of every NEE vertex within the recycling
 * radius (its own included) with its own BSDF and averages them; n_E in
 * eq. misw becomes the number of events found.  A light sample does not
 * depend on the receiving point (light by power, point uniform on it), so
 * only its visibility, tested from the vertex that drew it, is borrowed. */
static void recycled_nee(const o_iter* it, int vi, o_accum* acc) {
    const o_scene* s = it->s;
    const o_params* prm = it->prm;
    int p = it->v_path[vi], m = it->v_depth[vi];
    size_t id = IDX(it, p, m);
    v3 x = it->pos[id], n = it->nrml[id], wo = it->wo[id], tau = it->tau[id];
    const o_material* mt = &s->mats[it->mat[id]];
    if (mat_is_delta(mt)) return;
    double R2 = prm->nee_radius * prm->nee_radius, ne = it->v_ne[vi];
    double r2pi = PI * prm->merge_radius * prm->merge_radius;
    v3 sum = mk(0, 0, 0);
    for (int q = 0; q < it->nvert; ++q) {
        if (!it->v_lsok[q]) continue;
        v3 dq = sub(mk(it->v_pos[3 * q], it->v_pos[3 * q + 1], it->v_pos[3 * q + 2]), x);
        if (!(dot(dq, dq) < R2)) continue;
        const light_sample* L = &it->v_ls[q];
        v3 dv = sub(L->x, x);
        double d2 = dot(dv, dv);
        v3 w = scl(dv, 1.0 / sqrt(d2));
        double cx = fabs(dot(n, w));
        v3 dE, ln;
        if (L->tri >= 0) {
            double cl = -dot(L->n, w);
            if (!(cl > 0.0) || !(cx > 0.0)) continue;
            dE = scl(from_f(s->mats[s->mat[L->tri]].emission), cx * cl / (d2 * L->p_light));
            ln = L->n;
        } else {
            if (!(cx > 0.0)) continue;
            dE = scl(from_f(s->pl[L->pl].power), cx / (4.0 * PI * d2 * L->p_light));
            ln = scl(w, -1.0);
        }
        v3 f = bsdf_f(mt, n, wo, w);
        if (is_zero(f)) continue;
        o_path P;
        P.L = m + 1;
        path_from_camera(it, p, m, &P);
        P.seg_a[m] = x; P.seg_b[m] = L->x; P.na[m] = n; P.nb[m] = ln;
        P.p_light = L->p_light; P.hittable = L->hittable; P.rho = it->v_rho[vi]; P.r2pi = r2pi;
        P.photons = prm->enable_photons;
        P.n_lp = 0.0;
        P.n_e = ne;
        sum = add(sum, scl(hmul(hmul(tau, f), dE), mis_weight(&P, 1)));
    }
    add_px(acc->E, it->pixel[p], scl(sum, 1.0 / ne));
}

static void emission_event(const o_iter* it, int e, o_accum* acc) {
    const o_scene* s = it->s;
    int p = it->ev_path[e], l = it->ev_depth[e], tri = it->ev_tri[e];
    o_path P;
    P.L = l;
    path_from_camera(it, p, l, &P);
    P.p_light = s->light_psel[s->tri_light[tri]] / s->area[tri];
    P.hittable = 1;
    P.rho = 0.0;
    if (l >= 2) {
        size_t id = IDX(it, p, l - 1);
        P.rho = it->v_rho[it->vid[id]];
    }
    P.r2pi = PI * it->prm->merge_radius * it->prm->merge_radius;
    P.photons = it->prm->enable_photons;
    P.n_lp = it->prm->light_photons;
    P.n_e = l >= 2 ? it->v_ne[it->vid[IDX(it, p, l - 1)]] : 1.0;
    double w = mis_weight(&P, 0);
    add_px(acc->e, it->pixel[p], scl(it->ev_val[e], w));
}

/* pass 2 (d), optional conventional photons (Sec. 4, eq. stdphotonpdf):
 * light photon i of this iteration.  A light is picked by power and a
 * point on it as for NEE (stream LIGHT, word 0); the direction (word 1)
 * follows the cosine lobe of an area light or the uniform sphere of a
 * point light, so the emitted flux is L_e pi / p_light (area) or
 * power / P_sel (point), shared by the n_LP photons.  At every non-delta
 * hit y_j the view vertices within r of depth k with k + j <= maxlen
 * receive w_LP tau f Phi / (pi r^2).  The density rho at the first hit
 * (the start of the NEB technique for these paths) is queried once. */
static void light_photon(const o_iter* it, int i, int iter, o_accum* acc) {
    const o_scene* s = it->s;
    const o_params* prm = it->prm;
    if (s->nlights == 0) return;
    double u[4], u2[4];
    uniforms(it->key, (uint32_t)i, (uint32_t)iter, 0u, TAG_LIGHT, u);
    uniforms(it->key, (uint32_t)i, (uint32_t)iter, 1u, TAG_LIGHT, u2);
    int li = 0;
    while (li < s->nlights - 1 && !(u[0] < s->light_cdf[li])) ++li;
    double psel = s->light_psel[li];
    double nlp = (double)prm->light_photons;
    int L = prm->max_path_len;
    v3 ypos[MAXL], yn[MAXL];
    const o_material* ymat[MAXL];
    v3 o, d, phi;
    double p_light;
    int hittable;
    if (s->light_tri[li] >= 0) {
        int t = s->light_tri[li];
        double su = sqrt(u[1]);
        double b0 = 1.0 - su, b1 = u[2] * su;
        v3 y0 = add(add(scl(s->p0[t], b0), scl(s->p1[t], b1)), scl(s->p2[t], 1.0 - b0 - b1));
        v3 ln = s->ng[t], t1, t2;
        onb(ln, &t1, &t2);
        double rr = sqrt(u2[0]), ph = 2.0 * PI * u2[1], z = sqrt(fmax(0.0, 1.0 - u2[0]));
        d = nrm(add(add(scl(t1, rr * cos(ph)), scl(t2, rr * sin(ph))), scl(ln, z)));
        if (dot(d, ln) <= 0.0) return;
        p_light = psel / s->area[t];
        phi = scl(from_f(s->mats[s->mat[t]].emission), PI / (p_light * nlp));
        o = offset_origin(s, y0, ln, d);
        ypos[0] = y0; yn[0] = ln;
        hittable = 1;
    } else {
        const o_point_light* l = &s->pl[s->light_pl[li]];
        double z = 1.0 - 2.0 * u2[0], rr = sqrt(fmax(0.0, 1.0 - z * z)), ph = 2.0 * PI * u2[1];
        d = mk(rr * cos(ph), rr * sin(ph), z);
        p_light = psel;
        phi = scl(from_f(l->power), 1.0 / (psel * nlp));
        o = from_f(l->pos);
        ypos[0] = o; yn[0] = d;
        hittable = 0;
    }
    acc->st.light_photons += 1;
    double r = prm->merge_radius, r2pi = PI * r * r, rho1 = 0.0;
    for (int j = 1; j <= L - 1; ++j) {
        double t;
        int prim = closest_hit(s, o, d, &t);
        acc->st.rays += 1;
        if (prim < 0) break;
        acc->st.photon_segments += 1;
        v3 y = add(o, scl(d, t));
        v3 ny = s->ng[prim];
        const o_material* my = &s->mats[s->mat[prim]];
        ypos[j] = y; yn[j] = ny; ymat[j] = my;
        if (j == 1 && prm->enable_photons) rho1 = query_density(it, y, ny);
        if (!mat_is_delta(my)) {
            v3 wd = scl(d, -1.0);
            for (int q = 0; q < it->nvert; ++q) {
                int k = it->v_depth[q];
                if (k + j > L) continue;
                size_t qid = IDX(it, it->v_path[q], k);
                v3 dq = sub(it->pos[qid], y);
                if (dot(dq, dq) >= r * r) continue;
                const o_material* mq = &s->mats[it->mat[qid]];
                if (mat_is_delta(mq)) continue;
                v3 f = bsdf_f(mq, it->nrml[qid], it->wo[qid], wd);
                if (is_zero(f)) continue;
                o_path P;
                P.L = k + j;
                path_from_camera(it, it->v_path[q], k, &P);
                /* from the merge point (photon hit geometry) back along the photon to the light */
                P.seg_a[k] = y; P.seg_b[k] = ypos[j - 1]; P.na[k] = ny; P.nb[k] = yn[j - 1];
                for (int ii = 1; ii <= j - 1; ++ii) {
                    P.seg_a[k + ii] = ypos[j - ii]; P.seg_b[k + ii] = ypos[j - ii - 1];
                    P.na[k + ii] = yn[j - ii]; P.nb[k + ii] = yn[j - ii - 1];
                    P.mat[k + ii] = ymat[j - ii]; P.vn[k + ii] = yn[j - ii];
                }
                P.p_light = p_light; P.hittable = hittable; P.rho = rho1; P.r2pi = r2pi;
                P.photons = prm->enable_photons;
                P.n_lp = nlp;
                P.n_e = 1.0;
                double w = mis_weight(&P, lp_tech(P.L, k));
                add_px(acc->LP, it->pixel[it->v_path[q]], scl(hmul(hmul(it->tau[qid], f), phi), w / r2pi));
                acc->st.merges += 1;
            }
        }
        if (j == L - 1 || mat_is_black(my)) break;
        uniforms(it->key, (uint32_t)i, (uint32_t)iter, (uint32_t)(j - 1), TAG_PHOTON, u);
        bsdf_sample bs = sample_bsdf(my, ny, scl(d, -1.0), u);
        if (!bs.ok) break;
        phi = hmul(phi, bs.weight);
        o = offset_origin(s, y, ny, bs.dir);
        d = bs.dir;
    }
}

static int nthreads_of(const o_params* prm) {
#ifdef _OPENMP
    return prm->n_threads > 0 ? prm->n_threads : omp_get_max_threads();
#else
    (void)prm;
    return 1;
#endif
}

int32_t orc_render(const o_scene* s, const o_params* prm, int32_t n_iter, int32_t first_iter,
                   o_octree* oct, double* img_e, double* img_E, double* img_P, double* img_LP, o_stats* st,
                   o_record* rec) {
    if (!s || !prm || prm->width <= 0 || prm->height <= 0 || prm->max_path_len < 1 ||
        prm->max_path_len > MAXL - 2 || n_iter < 0)
        return -1;
    if ((prm->density_mode == 0 || prm->density_mode == 1) && !oct) return -1;
    if (prm->light_photons < 0) return -1;
    if (prm->nee_radius < 0.0 || (prm->nee_radius > 0.0 && prm->light_photons > 0)) return -1;
    if ((prm->density_mode == 4 || prm->density_mode == 5) &&
        (!(prm->density_radius > 0.0) || prm->knn_k < 1 || prm->knn_k > 64))
        return -1;
    const int L_lp = prm->max_path_len >= 2 ? prm->light_photons : 0;
    o_iter it;
    memset(&it, 0, sizeof(it));
    it.s = s; it.prm = prm; it.oct = oct;
    it.cam = make_cam(&s->cam, prm->width, prm->height);
    it.key.key[0] = (uint32_t)prm->seed;
    it.key.key[1] = prm->scene_id;
    it.L = prm->max_path_len;
    int x0 = prm->win_x0, y0 = prm->win_y0, x1 = prm->win_x1, y1 = prm->win_y1;
    if (x1 <= x0 || y1 <= y0) { x0 = 0; y0 = 0; x1 = prm->width; y1 = prm->height; }
    it.win_w = x1 - x0;
    it.npath = (x1 - x0) * (y1 - y0);
    size_t nslot = (size_t)it.npath * (size_t)(it.L + 1);
    it.pos = calloc(nslot, sizeof(v3)); it.nrml = calloc(nslot, sizeof(v3));
    it.wo = calloc(nslot, sizeof(v3)); it.tau = calloc(nslot, sizeof(v3));
    it.mat = calloc(nslot, sizeof(int)); it.prim = calloc(nslot, sizeof(int));
    it.vid = calloc(nslot, sizeof(int));
    it.nhit = calloc((size_t)it.npath, sizeof(int));
    it.pixel = calloc((size_t)it.npath, sizeof(int));
    it.v_path = calloc(nslot, sizeof(int)); it.v_depth = calloc(nslot, sizeof(int));
    it.v_rho = calloc(nslot, sizeof(double));
    it.v_pos = calloc(3 * nslot, sizeof(double));
    it.v_ne = calloc(nslot, sizeof(double));
    it.v_ls = calloc(nslot, sizeof(light_sample));
    it.v_lsok = calloc(nslot, sizeof(int));
    for (int yy = y0, p = 0; yy < y1; ++yy)
        for (int xx = x0; xx < x1; ++xx, ++p) it.pixel[p] = yy * prm->width + xx;
    int nth = nthreads_of(prm);
    size_t npix = (size_t)prm->width * (size_t)prm->height * 3;
    o_accum* acc = calloc((size_t)nth, sizeof(o_accum));
    for (int t = 0; t < nth; ++t) {
        acc[t].e = calloc(npix, sizeof(double));
        acc[t].E = calloc(npix, sizeof(double));
        acc[t].P = calloc(npix, sizeof(double));
        acc[t].LP = calloc(npix, sizeof(double));
    }
    memset(st, 0, sizeof(*st));
    for (int32_t ii = 0; ii < n_iter; ++ii) {
        int iter = first_iter + ii;
        const int frozen = prm->freeze_after > 0 && iter > prm->freeze_after;
        if (oct && !frozen) orc_octree_set_iteration(oct, iter);
        memset(it.vid, 0, nslot * sizeof(int));
        it.nev = 0;
        o_record* r = (rec && ii == 0) ? rec : NULL;
        if (r) memset(r, 0, sizeof(o_record) * (size_t)it.npath * (size_t)it.L);
        /* pass 1 */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
#endif
        for (int p = 0; p < it.npath; ++p) trace_camera_path(&it, p, iter, r);
        /* canonical vertex order: depth-major, then pixel */
        it.nvert = 0;
        for (int k = 1; k <= it.L - 1; ++k)
            for (int p = 0; p < it.npath; ++p) {
                size_t id = IDX(&it, p, k);
                if (it.vid[id]) {
                    it.vid[id] = it.nvert;
                    it.v_path[it.nvert] = p; it.v_depth[it.nvert] = k;
                    it.nvert++;
                } else {
                    it.vid[id] = -1;
                }
            }
        /* deposits, sequential in canonical order */
        if (oct && !frozen) {
            for (int q = 0; q < it.nvert; ++q) {
                v3 x = it.pos[IDX(&it, it.v_path[q], it.v_depth[q])];
                float f[3] = {(float)x.x, (float)x.y, (float)x.z};
                octree_insert(oct, f);
            }
        }
        for (int q = 0; q < it.nvert; ++q) {
            v3 x = it.pos[IDX(&it, it.v_path[q], it.v_depth[q])];
            it.v_pos[3 * q] = x.x; it.v_pos[3 * q + 1] = x.y; it.v_pos[3 * q + 2] = x.z;
        }
        /* pass 2 (a): densities */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
#endif
        for (int q = 0; q < it.nvert; ++q) {
            size_t id = IDX(&it, it.v_path[q], it.v_depth[q]);
            it.v_rho[q] = query_density(&it, it.pos[id], it.nrml[id]);
        }
        if (prm->density_hook && it.nvert > 0) {
            double* hp = malloc(sizeof(double) * 6 * (size_t)it.nvert);
            int32_t* hi = malloc(sizeof(int32_t) * 2 * (size_t)it.nvert);
            for (int q = 0; q < it.nvert; ++q) {
                size_t id = IDX(&it, it.v_path[q], it.v_depth[q]);
                v3 x = it.pos[id], nn = it.nrml[id];
                hp[3 * q] = x.x; hp[3 * q + 1] = x.y; hp[3 * q + 2] = x.z;
                double* hn = hp + 3 * (size_t)it.nvert;
                hn[3 * q] = nn.x; hn[3 * q + 1] = nn.y; hn[3 * q + 2] = nn.z;
                hi[q] = it.pixel[it.v_path[q]];
                hi[it.nvert + q] = it.v_depth[q];
            }
            prm->density_hook(it.nvert, hp, hp + 3 * (size_t)it.nvert, hi, hi + it.nvert, iter, it.v_rho);
            free(hp);
            free(hi);
        }
        /* n_E: the NEE events each vertex will use (recycling: all NEE
         * vertices within the radius, the vertex itself included) */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
#endif
        for (int q = 0; q < it.nvert; ++q) {
            it.v_ne[q] = 1.0;
            if (prm->nee_radius > 0.0) {
                double R2 = prm->nee_radius * prm->nee_radius, c = 0.0;
                for (int j = 0; j < it.nvert; ++j) {
                    double dx = it.v_pos[3 * j] - it.v_pos[3 * q], dy = it.v_pos[3 * j + 1] - it.v_pos[3 * q + 1];
                    double dz = it.v_pos[3 * j + 2] - it.v_pos[3 * q + 2];
                    if (dx * dx + dy * dy + dz * dz < R2) c += 1.0;
                }
                it.v_ne[q] = c;
            }
        }
        /* pass 2 (b, c): NEE and photons */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 8) num_threads(nth)
#endif
        for (int q = 0; q < it.nvert; ++q) {
#ifdef _OPENMP
            int t = omp_get_thread_num();
#else
            int t = 0;
#endif
            nee_and_photon(&it, q, iter, &acc[t]);
        }
        /* pass 2 (b'): NEE recycling */
        if (prm->nee_radius > 0.0) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
#endif
            for (int q = 0; q < it.nvert; ++q) {
#ifdef _OPENMP
                int t = omp_get_thread_num();
#else
                int t = 0;
#endif
                recycled_nee(&it, q, &acc[t]);
            }
        }
        /* pass 2 (d): conventional light photons */
        if (L_lp > 0) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 8) num_threads(nth)
#endif
            for (int i = 0; i < L_lp; ++i) {
#ifdef _OPENMP
                int t = omp_get_thread_num();
#else
                int t = 0;
#endif
                light_photon(&it, i, iter, &acc[t]);
            }
        }
        /* pass 3 */
        for (int e = 0; e < it.nev; ++e) emission_event(&it, e, &acc[0]);
        st->paths += it.npath;
        st->vertices += it.nvert;
        st->events += it.nev;
        for (int p = 0; p < it.npath; ++p) st->rays += it.nhit[p] + (it.nhit[p] < it.L ? 1 : 0);
    }
    for (int t = 0; t < nth; ++t) {
        for (size_t i = 0; i < npix; ++i) {
            if (img_e) img_e[i] += acc[t].e[i];
            if (img_E) img_E[i] += acc[t].E[i];
            if (img_P) img_P[i] += acc[t].P[i];
            if (img_LP) img_LP[i] += acc[t].LP[i];
        }
        st->photons += acc[t].st.photons;
        st->photon_segments += acc[t].st.photon_segments;
        st->merges += acc[t].st.merges;
        st->nee_visible += acc[t].st.nee_visible;
        st->rays += acc[t].st.rays;
        st->light_photons += acc[t].st.light_photons;
        free(acc[t].e); free(acc[t].E); free(acc[t].P); free(acc[t].LP);
    }
    free(acc);
    if (oct) {
        int64_t info[8];
        orc_octree_export(oct, NULL, 0, info);
        st->oct_capacity = info[0]; st->oct_nodes = info[1]; st->oct_depth = info[2];
        st->oct_ledger = info[3]; st->oct_deposits = info[4]; st->oct_overflow = info[5];
        st->oct_rejected = info[6];
    }
    free(it.pos); free(it.nrml); free(it.wo); free(it.tau); free(it.mat); free(it.prim);
    free(it.vid); free(it.nhit); free(it.pixel); free(it.v_path); free(it.v_depth); free(it.v_rho); free(it.v_pos);
    free(it.v_ne); free(it.v_ls); free(it.v_lsok);
    free(it.ev_path); free(it.ev_depth); free(it.ev_tri); free(it.ev_val);
    return 0;
}

/* ------------------------------------------------------------------ */
/* MIS test hook: densities of all techniques of an explicit path       */
/* ------------------------------------------------------------------ */
/* pos: (L+1) x 3 vertex positions (camera first, light last); nrmv: the
 * same for normals (camera normal unused; at the light, its normal, used
 * for an area light's emission cosine); mats: materials of vertices
 * 1..L-1; n_lp: light photons per iteration.  out holds 2 L entries:
 * e, E, P_1 .. P_{L-2}, LP_1 .. LP_{L-1}.  Returns the number of
 * techniques written (2 + max(0, L-2) + max(0, L-1)). */
int32_t orc_path_technique_densities(int32_t L, const double* pos, const double* nrmv,
                                     const o_material* mats, double p_light, int32_t hittable,
                                     double rho, double radius, int32_t photons, double n_lp,
                                     double* out) {
    if (L < 1 || L > MAXL - 2) return 0;
    o_path P;
    memset(&P, 0, sizeof(P));
    P.L = L;
    for (int i = 0; i < L; ++i) {
        P.seg_a[i] = mk(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
        P.seg_b[i] = mk(pos[3 * i + 3], pos[3 * i + 4], pos[3 * i + 5]);
        P.na[i] = mk(nrmv[3 * i], nrmv[3 * i + 1], nrmv[3 * i + 2]);
        P.nb[i] = mk(nrmv[3 * i + 3], nrmv[3 * i + 4], nrmv[3 * i + 5]);
    }
    for (int i = 1; i <= L - 1; ++i) {
        P.mat[i] = &mats[i - 1];
        P.vn[i] = mk(nrmv[3 * i], nrmv[3 * i + 1], nrmv[3 * i + 2]);
    }
    P.p_light = p_light; P.hittable = hittable; P.rho = rho;
    P.r2pi = PI * radius * radius; P.photons = photons; P.n_lp = n_lp; P.n_e = 1.0;
    path_densities(&P, out);
    return n_techniques(L);
}
