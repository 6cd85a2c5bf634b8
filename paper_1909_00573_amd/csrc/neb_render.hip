// Wavefront Next Event Backtracking on gfx950.
//
// One iteration (one sample per pixel) runs the three passes of Sec. 3:
//   pass 1  camera -> [extend -> shade] x maxlen: view paths, NEE-vertex
//           store, emitter-hit events, compaction of live paths;
//           octree deposits of every NEE vertex (Sec. 5.1, 5.2)
//   pass 2  density per vertex (eq. octdensity, robust query) -> NEE with the
//           shadow ray, L_E, and the photon of flux dE / rho (eq. flux) with
//           its first scatter at the vertex -> merge grid over the view
//           vertices -> [extend -> merge + scatter] x (maxlen - 2)
//           optional conventional light photons (Sec. 4): emitted from the
//           lights before the NEB photons enter the same queue, their first
//           hit gets its density, then they share the merge loop
//   pass 3  emitter-hit events weighted with w_e (Sec. 3.3)
// MIS weights (Sec. 4, balance heuristic over e, E, P_k and, with light
// photons, LP_k) are evaluated with running ratios carried by the view and
// photon states, so no event needs the full path: each view vertex stores
// B = A_{m-2} + [x_{m-1} not delta] and g = |cos out at x_{m-1}| / (pdf at
// x_{m-1} * |cos in at x_m|), each photon carries U and h with the same
// meaning from the light side.  The light-photon terms of eq. misw sum to
// n_LP pi r^2 p_{l -> l-1} (A_{l-2} + [x_{l-1} not delta]); a photon folds
// the constant factor they add to its merges into its flux and its U.
//
// A context holds a batch of 1..256 scenes that share every pool: a BVH
// forest (one root per scene in one node pool), one octree node pool split
// into per-scene ranges, one set of queues and one merge grid whose key
// includes the scene.  Every launch covers all scenes; each state word
// carries its scene in bits 8..15.  Random numbers are drawn with the
// scene-local pixel and the scene's key, so a scene renders the same paths
// in a batch as alone.  The iteration number and the octree's iteration
// scalars live in device memory, so one captured iteration (a hipGraph)
// replays for every iteration.
#include <algorithm>
#include <chrono>
#include <random>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "neb_bvh.h"
#include "neb_device.h"
#include "neb_mlp.h"

namespace neb {

constexpr int kMaxScenes = 256;
constexpr int kMaxMaterials = 65536;

// ---------------------------------------------------------------------------
// state layouts (SoA of float4, ints stored as float bits; "tag" words hold
// a depth code in bits 0..7, the scene in bits 8..15 and, for vertices, the
// global material id in bits 16..31)
//   path q0 (o.xyz, global pixel)  q1 (d.xyz, tag: depth of the next hit)
//        q2 (tau.rgb, pdf of the sampled direction at the last vertex)
//        q3 (A_{m-1}, |cos out|/pdf at the last vertex, last vertex non-delta, last vertex index)
//   vertex v0 (pos, global pixel)  v1 (n, tag: depth | scene | material)  v2 (wo, B)  v3 (tau, g)
//   event e0 (tau*Le, p_light/f or 0 for a direct hit)
//         e1 (pi r^2 A, prev non-delta + light-photon term, prev vertex, global pixel)
//   photon p0 (o, global origin pixel)  p1 (d, tag: 16*origin depth + bounce)
//          p2 (Phi, |cos out|/pdf)  pu (U)
//          a light photon has origin depth 0 and p0.w = its scene's first
//          pixel + its index; before its first hit pu holds its light, at
//          its first hit p2.w and pu hold its MIS terms (k_lp_first)
// ---------------------------------------------------------------------------
struct PathQ {
    float4 *q0, *q1, *q2, *q3;
};
struct PhotonQ {
    float4 *p0, *p1, *p2;
    float* pu;
};
struct VertexStore {
    float4 *v0, *v1, *v2, *v3;
    float* rho;
    float* ne;       // NEE recycling: n_E, the NEE vertices within the radius (null: 1)
    float4* lsrec;   // NEE recycling: each vertex's light point and light (-1: no contribution)
};
struct Images {
    float *e, *E, *P, *LP;
};

// per-scene constants, one entry per scene of the batch (device array)
struct SceneInfo {
    CamParams cam;
    int32_t pix_base;   // first global pixel of the scene
    int32_t npix;
    int32_t L;          // maximum path length
    int32_t spp;        // iterations the scene takes part in (0 = all)
    int32_t bvh_root;   // root node of the scene's tree in the forest
    int32_t light_base; // first light of the scene in the light pool
    int32_t n_lights;
    int32_t pad;
    uint32_t k0, k1;    // Philox key
    float eps;          // ray offset
    float r, r2pi;      // merge radius and pi r^2
    float inv_cell;     // 1 / merge-grid cell size
    float rho0, cam_w;  // analytic density (test hook)
    int32_t n_lp;       // light photons per iteration
    int32_t lp_base;    // first global light-photon index of the scene
    float nlp;          // n_LP as a float (0: no light photons)
    float dr;           // density radius (modes 4, 5)
    float inv_dcell;    // 1 / density-grid cell size
    int32_t knn_k;      // k (mode 5)
    float nee_r;        // NEE recycling radius (0: off)
    float inv_ncell;    // 1 / recycling-grid cell size
    int32_t pad4;
};

// Merge grid keyed by (hash of scene and cell, depth class): the records of
// one cell are ordered by view-vertex depth class (depth - 1, the last of
// the D classes also holding every deeper vertex), so the vertices a photon
// after j bounces may merge with (depth <= maxlen - 1 - j) lie in one
// contiguous prefix; only the last class's deeper vertices are filtered by
// the depth each entry carries.
struct Grid {
    int32_t* count;   // T * D + 1 entries (the last stays 0); zeroed by the scan that reads them
    int32_t* start;   // T * D + 1 entries
    int32_t* rank;    // per view vertex: its place among the vertices of its key
    float4* sorted;   // (pos, scene | depth << 24) in (cell, depth class) order
    float4* mrec;     // 4 per record, same order: what a merge needs of the view vertex:
                      // (n, tag), (wo, B), (tau, g), (pixel, -, -, -)
    int32_t* sums;    // scan block sums, all levels
    int32_t T;        // hash buckets (power of two)
    int32_t D;        // depth classes: 8 (a cell's row is one aligned 32-byte sector)
};

// prefix sums are scanned in tiles of kScanTile elements (a tile per block
// of kScanBlock threads, kScanPer each)
constexpr int kScanPer = 16;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanPer * kScanBlock;


// Density grid of the alternative providers: every NEE vertex of the
// iteration, keyed by the hash of its scene and its cell of size
// 2 * density radius (so a query ball touches at most 8 cells).
struct DGrid {
    int32_t* count;   // T + 1 entries (the last stays 0)
    int32_t* start;   // T + 1 entries
    float4* pts;      // (pos, scene) in bucket order
    int32_t* vidx;    // vertex index of each entry (NEE recycling grid only)
    int32_t* sums;    // scan block sums
    int32_t T;        // buckets (power of two)
};

struct RenderArgs {
    SceneView S;
    const SceneInfo* sc;
    const int32_t* pix_base;  // n_scenes + 1 entries
    Counters* cnt;
    int32_t n_scenes;
    int32_t L;                // longest maximum path length of the batch
    int32_t npix;             // pixels of all scenes
    int32_t photons;          // n_P > 0
    int32_t density_mode;
    const int32_t* lp_base;   // n_scenes + 1 entries: light photons of the scenes before
    int32_t n_lp;             // light photons of all scenes per iteration
    DGrid dg;                 // NEB_DENSITY_RADIUS / NEB_DENSITY_KNN
    DGrid ng;                 // NEE recycling: the NEE vertices by cells of 2 * recycling radius
    int32_t recycle;          // NEE recycling on
};

__device__ __forceinline__ int fbits(float f) { return __float_as_int(f); }
__device__ __forceinline__ float ibits(int i) { return __int_as_float(i); }
__device__ __forceinline__ int tag_depth(int w) { return w & 0xFF; }
__device__ __forceinline__ int tag_scene(int w) { return (w >> 8) & 0xFF; }
__device__ __forceinline__ int tag_mat(int w) { return (int)((uint32_t)w >> 16); }
__device__ __forceinline__ int make_tag(int depth, int scene) { return depth | (scene << 8); }
__device__ __forceinline__ int make_vtag(int depth, int scene, int mat) { return depth | (scene << 8) | (mat << 16); }

__device__ __forceinline__ bool scene_active(const SceneInfo& I, int iter) { return I.spp == 0 || iter <= I.spp; }

__device__ __forceinline__ f3 offset_origin(f3 x, f3 n, f3 dir, float eps) {
    return dot3(dir, n) > 0.f ? x + n * eps : x - n * eps;
}

__device__ __forceinline__ void atomic_add3(float* img, int pixel, f3 c) {
    float* p = img + 3 * (size_t)pixel;
    atomicAdd(p, c.x);
    atomicAdd(p + 1, c.y);
    atomicAdd(p + 2, c.z);
}

__device__ __forceinline__ f3 cam_ray(const CamParams& C, int px, int py, float u0, float u1) {
    float sx = (2.0f * ((float)px + u0) / (float)C.w - 1.0f) * C.tan_half * C.aspect;
    float sy = (1.0f - 2.0f * ((float)py + u1) / (float)C.h) * C.tan_half;
    f3 f = load3(C.f), r = load3(C.r), u = load3(C.u);
    return normalize3(f + r * sx + u * sy);
}

// primary-hit density per unit area of the pinhole camera (test density hook)
__device__ __forceinline__ float cam_hit_density(const CamParams& C, f3 x, f3 n) {
    f3 d = x - load3(C.eye);
    float d2 = dot3(d, d);
    f3 w = d * rsqrtf(d2);
    float c = dot3(w, load3(C.f));
    if (c <= 0.f) return 0.f;
    float sx = dot3(w, load3(C.r)) / c, sy = dot3(w, load3(C.u)) / c;
    if (fabsf(sx) > C.tan_half * C.aspect || fabsf(sy) > C.tan_half) return 0.f;
    float film = 4.0f * C.tan_half * C.tan_half * C.aspect;
    return (float)C.w * (float)C.h / (film * c * c * c) * fabsf(dot3(n, w)) / d2;
}

// scene of a global pixel (or light photon): the last s with pix_base[s] <= i
__device__ __forceinline__ int scene_of_pixel(const int32_t* pix_base, int n_scenes, int i) {
    int lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pix_base[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
// Starts an iteration: advances the device iteration counter, sets the
// octree's iteration scalars (Appendix B set_iteration) and empties the
// queues.  The octree counts iterations 1..freeze only (freeze is the
// number of training iterations of the learned density, else unbounded).
__global__ void k_iter_begin(Counters* c, OctDyn* dyn, int32_t freeze) {
    int it = c->iter + 1;
    c->iter = it;
    for (int b = 0; b < kPhotonBufs; ++b) c->pcount[b] = 0;
    c->n_shadow = 0;
    c->lp_count = 0;
    int oit = it < freeze ? it : freeze;
    int ic = oit < kOctFillIterations ? oit : kOctFillIterations;
    OctDyn d;
    d.iter = oit;
    d.split_count = kOctSplitFactor * ic;
    d.density_scale = 1.0f / (float)ic;
    d.stop_filling = it > kOctFillIterations || it > freeze;
    *dyn = d;
}
__global__ void k_iter_end(Counters* c, int parity) {
    c->st[0].vertices += (unsigned long long)c->n_vertices[parity];
    c->st[0].events += (unsigned long long)c->n_events[parity];
}
// Starts the camera pass of an iteration (it may run while the iteration
// before still bounces photons): its own iteration counter, the path queues
// and the vertex and event stores of its parity emptied.
__global__ void k_cam_begin(Counters* c, int parity) {
    c->iter_cam += 1;
    c->qcount[0] = 0;
    c->qcount[1] = 0;
    c->n_vertices[parity] = 0;
    c->n_events[parity] = 0;
}
__global__ void k_mean_image(const float* e, const float* E, const float* P, const float* LP, float* out, int64_t n,
                             float scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (e[i] + E[i] + P[i] + LP[i]) * scale;
}
__global__ void k_scale_image(const float* a, float* out, int64_t n, float scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] * scale;
}

// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
// one camera ray per pixel of every scene still taking part; the live rays
// are compacted into the queue
// camera rays of the scenes active in this iteration, queue slots reserved
// once per block of kCameraBlock threads
constexpr int kCameraBlock = 512;
__global__ void __launch_bounds__(kCameraBlock) k_camera(RenderArgs A, PathQ q) {
    __shared__ int wc[kCameraBlock / 64];
    __shared__ int bb;
    const int iter = A.cnt->iter_cam;
    unsigned started = 0;
    for (int base = blockIdx.x * kCameraBlock; base < A.npix; base += gridDim.x * kCameraBlock) {
        const int i = base + threadIdx.x;
        int s = i < A.npix ? scene_of_pixel(A.pix_base, A.n_scenes, i) : 0;
        const SceneInfo& I = A.sc[s];
        bool act = i < A.npix && scene_active(I, iter);
        int slot = block_reserve<kCameraBlock / 64>(&A.cnt->qcount[0], act, wc, &bb);
        if (act) {
            int local = i - I.pix_base;
            int px = local % I.cam.w, py = local / I.cam.w;
            U4 u = uniforms(I.k0, I.k1, (uint32_t)local, (uint32_t)iter, 0u, kTagCamera);
            f3 d = cam_ray(I.cam, px, py, u.u[0], u.u[1]);
            q.q0[slot] = f4(load3(I.cam.eye), ibits(i));
            q.q1[slot] = f4(d, ibits(make_tag(1, s)));
            q.q2[slot] = make_float4(1.f, 1.f, 1.f, 0.f);
            q.q3[slot] = make_float4(0.f, 0.f, 0.f, ibits(-1));
            ++started;
        }
    }
    wave_add_u64(&stat_line(A.cnt).paths, started);
}

// Spatial bins of photon hits: a 2^bits-per-axis grid over each scene's
// octree box in Morton order (neighbouring bins are neighbouring boxes),
// scenes one after another, and one last bin for the rays that missed.
struct HitBins {
    int32_t* bin;          // per ray: its bin (null: no binning)
    int32_t* count;        // per bin: rays (returns to zero after the scatter)
    const OctParams* prm;  // per scene: the box
    int32_t bits;          // per axis
    int32_t n_bins;        // bins of all scenes; the miss bin is n_bins
};

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // bits b -> 3b
    v &= 0x3FF;
    v = (v | (v << 16)) & 0x030000FF;
    v = (v | (v << 8)) & 0x0300F00F;
    v = (v | (v << 4)) & 0x030C30C3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

__device__ __forceinline__ int hit_bin(const HitBins& B, int scene, f3 y) {
    const OctParams& P = B.prm[scene];
    const float res = (float)(1 << B.bits);
    float v[3] = {y.x, y.y, y.z};
    uint32_t c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float q = (v[k] - P.min_bound[k]) * P.size_inv[k];
        c[k] = (uint32_t)min((int)res - 1, max(0, (int)(q * res)));
    }
    return (scene << (3 * B.bits)) + (int)(spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2));
}

// closest hit for a queue of rays given as (origin, direction) float4 arrays
// (the direction's w is a tag word naming the scene); also clears the
// counter of the queue the next kernel appends to (if any).  kAnyHit: shadow
// rays, each ending at tmax[i]; vis[origin's w word] gets 1 if nothing is
// hit before it, else 0 (no hits are written).  ray_kind names the statistic
// the rays count in: 0 camera, 1 photon, 2 shadow rays.  Optionally counts
// the hits per spatial bin
template <int kStack, bool kAnyHit>
__global__ void __launch_bounds__(kTraceBlock) k_extend(SceneView S, const SceneInfo* sc,
                                                        const float4* __restrict__ org,
                                                        const float4* __restrict__ dir, const int32_t* count,
                                                        int32_t* next_count, int2* __restrict__ hits,
                                                        int ray_kind, Counters* cnt, HitBins B,
                                                        const float* __restrict__ tmax, int32_t* __restrict__ vis,
                                                        WorkLine* work, int32_t* work_done) {
    __shared__ int stack[kStack * kTraceBlock];
    const int n = *count;
    if (next_count && blockIdx.x == 0 && threadIdx.x == 0) *next_count = 0;
    unsigned traced = 0, nodes = 0, tris = 0;
    // Each lane holds one ray; a lane whose ray ends takes the next one from
    // a work counter (one atomic per wave), so short rays do not leave lanes
    // idle behind long ones.  The queue is cut into chunks of kChunk rays
    // dealt round-robin to `parts` parts, each with a counter of its own;
    // block b draws from part b mod parts (blocks b, b + 8, ... share an
    // XCD), so the counters' atomics are spread over eight cache lines while
    // every part's rays stay spread over the whole queue.
    constexpr int kSteps = 16;  // node visits per round (four-wide nodes: 16 beats 32 by 1-3 %)
    constexpr int kChunk = 256;
    const int parts = min(kWorkParts, (int)gridDim.x), part = blockIdx.x % parts;
    int32_t* next = &work[part].next;
    int i = -1;  // this lane's ray; >= n once the queue is exhausted
    TraceState T;
    f3 o = mk3(0.f, 0.f, 0.f), dd = mk3(0.f, 0.f, 1.f);
    int sid = 0;
    for (;;) {
        const bool need = i < 0;
        const int got = wave_reserve(next, need);
        if (need) {
            const int64_t g = ((int64_t)(got / kChunk) * parts + part) * kChunk + got % kChunk;
            i = g < n ? (int)g : n;
            if (i < n) {
                float4 d4 = dir[i];
                sid = tag_scene(fbits(d4.w));
                o = xyz(org[i]);
                dd = xyz(d4);
                trace_begin(T, sc[sid].bvh_root, o, dd, kAnyHit ? tmax[i] : INFINITY);
            }
        }
        const bool act = i < n;
        if (!__any(act)) break;
        if (act && trace_steps<kStack, kAnyHit>(S, T, stack + threadIdx.x, kSteps, nodes, tris)) {
            if (kAnyHit) {
                vis[fbits(org[i].w)] = T.prim < 0 ? 1 : 0;
            } else {
                hits[i] = make_int2(fbits(T.best), T.prim);
            }
            if (!kAnyHit && B.bin) {
                int b = T.prim >= 0 ? hit_bin(B, sid, o + dd * T.best) : B.n_bins;
                B.bin[i] = b;
                atomicAdd(&B.count[b], 1);
            }
            ++traced;
            i = -1;
        }
    }
    // the last block to finish resets the work counter for the next launch
    __syncthreads();
    if (threadIdx.x == 0 && atomicAdd(work_done, 1) == (int)gridDim.x - 1) {
        for (int k = 0; k < kWorkParts; ++k) work[k].next = 0;
        *work_done = 0;
    }
    StatLine& L = stat_line(cnt);
    wave_add_u64(ray_kind == 0 ? &L.camera_rays : (ray_kind == 1 ? &L.photon_rays : &L.shadow_rays), traced);
    wave_add_u64(&L.bvh_nodes[ray_kind], nodes);
    wave_add_u64(&L.bvh_tris[ray_kind], tris);
}

// One thread per path.  The three appends (emitter event, NEE vertex,
// continuing path) are reserved once per block and queue: the eight waves'
// counts meet in LDS and one thread per queue takes the block's slots with
// one atomic, eight times fewer than one per wave (returning atomics on one
// counter are serialised).  Every thread runs the same number of rounds so
// that the block can meet at its barriers.  Blocks of 512 threads: larger
// ones wait longer for a CU with room beside the other streams' kernels,
// smaller ones take more atomics.
constexpr int kShadeBlock = 512;
__global__ void __launch_bounds__(kShadeBlock) k_shade(RenderArgs A, PathQ in, const int32_t* count_in,
                                                       const int2* hits, PathQ out, int32_t* count_out,
                                                       VertexStore V, int32_t* n_vertices, float4* ev0, float4* ev1,
                                                       int32_t* n_events, int32_t* slots, neb_path_record* rec) {
    constexpr int kWaves = kShadeBlock / 64;
    __shared__ int wc[3][kWaves];  // per queue and wave: appends of this round
    __shared__ int bb[3];          // per queue: the block's first slot
    const int n = *count_in;
    const SceneView& S = A.S;
    const int iter = A.cnt->iter_cam;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int base = blockIdx.x * kShadeBlock; base < n; base += gridDim.x * kShadeBlock) {
        const int i = base + threadIdx.x;
        const bool valid = i < n;
        float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0, a2 = a0, a3 = a0;
        int2 h = make_int2(0, -1);
        if (valid) {
            a0 = in.q0[i];
            a1 = in.q1[i];
            a2 = in.q2[i];
            a3 = in.q3[i];
            h = hits[i];
        }
        int pixel = fbits(a0.w), tg = fbits(a1.w);
        int k = tag_depth(tg), sid = tag_scene(tg);
        const SceneInfo& I = A.sc[sid];
        neb_path_record* rc = (rec && valid) ? rec + (size_t)pixel * A.L + (k - 1) : nullptr;
        bool alive = valid && h.y >= 0;
        if (valid && !alive && rc) {
            rc->type = 5;
            rc->mat = -1;
            rc->prim = -1;
        }
        int prim = h.y;
        float t = ibits(h.x);
        f3 o = xyz(a0), d = xyz(a1), tau = xyz(a2);
        f3 x = o + d * t;
        float4 pn = alive ? S.prim_n[prim] : make_float4(0.f, 0.f, 1.f, 0.f);
        f3 nrm = xyz(pn);
        int mid = fbits(pn.w);
        const neb_material& m = S.mats[alive ? mid : 0];
        f3 wo = -d;
        float cin = dot3(nrm, wo);
        if (alive && rc) {
            rc->type = 4;
            rc->mat = mid;
            rc->prim = prim;
            rc->pos[0] = x.x;
            rc->pos[1] = x.y;
            rc->pos[2] = x.z;
        }
        // emitter hit: stored for pass 3 (its MIS weight needs rho at x_{l-1})
        const bool emit = alive && mat_emits(m) && cin > 0.f && S.prim_light[prim] >= 0;
        const bool store = alive && !mat_black(m) && k <= I.L - 1;
        float g = (k >= 2) ? a3.y / fabsf(cin) : 0.f;
        float B = (k >= 2) ? a3.x + a3.z : 0.f;
        Sample smp;
        smp.ev = 0;
        if (store) {
            U4 u = uniforms(I.k0, I.k1, (uint32_t)(pixel - I.pix_base), (uint32_t)iter, (uint32_t)k, kTagBsdf);
            smp = bsdf_sample(m, nrm, wo, u);
        }
        const bool go = smp.ev != 0;
        if (go && rc) rc->type = smp.ev;
        // the block's slots in the three queues
        const unsigned long long me = __ballot(emit), ms = __ballot(store), mg = __ballot(go);
        if (lane == 0) {
            wc[0][wid] = __popcll(me);
            wc[1][wid] = __popcll(ms);
            wc[2][wid] = __popcll(mg);
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            const int q = threadIdx.x;
            int tot = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) tot += wc[q][w];
            int32_t* ctr = q == 0 ? n_events : (q == 1 ? n_vertices : count_out);
            bb[q] = tot ? atomicAdd(ctr, tot) : 0;
        }
        __syncthreads();
        int pe = bb[0], ps = bb[1], pg = bb[2];
        for (int w = 0; w < wid; ++w) {
            pe += wc[0][w];
            ps += wc[1][w];
            pg += wc[2][w];
        }
        __syncthreads();  // wc and bb are rewritten by the next round
        if (emit) {
            const int eslot = pe + __popcll(me & below);
            float q = 0.f, D = a3.z;
            if (k > 1) {
                int lid = S.prim_light[prim];
                float p_light = S.lights[5 * lid].w / S.lights[5 * lid + 1].w;
                float f_prev = a2.w * cin / (t * t);
                q = p_light / f_prev;
                // light photons: n_LP pi r^2 p_{l -> l-1} (A_{l-2} + delta_{l-1}), where the
                // emission density p_{l -> l-1} = (cin / pi) |cos out| / t^2 = (a3.y / pi) f_prev
                D += I.nlp * I.r * I.r * a3.y * f_prev * (a3.x + a3.z);
            }
            ev0[eslot] = f4(tau * load3(m.emission), q);
            ev1[eslot] = make_float4(a3.x * I.r2pi, D, a3.w, ibits(pixel));
        }
        const int vid = store ? ps + __popcll(ms & below) : -1;
        if (store) {
            V.v0[vid] = f4(x, ibits(pixel));
            V.v1[vid] = f4(nrm, ibits(make_vtag(k, sid, mid)));
            V.v2[vid] = f4(wo, B);
            V.v3[vid] = f4(tau, g);
            if (slots) slots[(size_t)(k - 1) * A.npix + pixel] = vid;
        }
        if (go) {
            const int slot = pg + __popcll(mg & below);
            float Acur = (k >= 2) ? bsdf_pdf(m, nrm, smp.dir, wo) * g * B : 0.f;
            float gp = fabsf(dot3(nrm, smp.dir)) / smp.pdf;
            float dnon = mat_delta(m.type) ? 0.f : 1.f;
            out.q0[slot] = f4(offset_origin(x, nrm, smp.dir, I.eps), ibits(pixel));
            out.q1[slot] = f4(smp.dir, ibits(make_tag(k + 1, sid)));
            out.q2[slot] = f4(tau * smp.w, smp.pdf);
            out.q3[slot] = make_float4(Acur, gp, dnon, ibits(vid));
        }
    }
}

// ---------------------------------------------------------------------------
// pass 2 (a): density at every NEE vertex
// ---------------------------------------------------------------------------
// Bucket of a cell: the cells of one 4 x 4 x 4 block take 64 consecutive
// buckets (Morton order inside the block), the blocks are hashed with the
// scene.  The <= 8 cells around a photon hit, and the cells of neighbouring
// hits, then share a few cache lines of the count/start tables.
__device__ __forceinline__ uint32_t cell_hash(int cx, int cy, int cz, int scene, int32_t T) {
    const uint32_t lo = (uint32_t)((cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2) | ((cx & 2) << 2) | ((cy & 2) << 3) |
                                   ((cz & 2) << 4));
    const uint32_t hi = ((uint32_t)(cx >> 2) * 73856093u) ^ ((uint32_t)(cy >> 2) * 19349663u) ^
                        ((uint32_t)(cz >> 2) * 83492791u) ^ ((uint32_t)scene * 2654435761u);
    return ((hi << 6) | lo) & (uint32_t)(T - 1);
}
__device__ __forceinline__ uint32_t point_hash(f3 p, float inv_cell, int scene, int32_t T) {
    return cell_hash((int)floorf(p.x * inv_cell), (int)floorf(p.y * inv_cell), (int)floorf(p.z * inv_cell), scene, T);
}

// Fixed-radius count (mode 4), k-th-neighbour distance (mode 5) or the bare
// number of points within R (mode 0) at x over
// the points of scene s in the density grid: the buckets of the <= 8 cells
// the ball of radius R touches (a bucket counted once even when two cells
// share it; points of other cells or scenes in a bucket fail the tests).
// Mode 5 keeps the 16 smallest squared distances in registers, sorted, by a
// min/max pass over all of them per point.
constexpr int kKnnMax = 16;
__device__ __forceinline__ float set_density(const DGrid& D, int s, f3 x, float R, float inv_cell, int mode, int k) {
    const float R2 = R * R;
    float best[kKnnMax];
#pragma unroll
    for (int t = 0; t < kKnnMax; ++t) best[t] = 3.0e38f;
    int m = 0;
    const float rr = R * 1.00001f;
    const int lx = (int)floorf((x.x - rr) * inv_cell), hx = min((int)floorf((x.x + rr) * inv_cell), lx + 1);
    const int ly = (int)floorf((x.y - rr) * inv_cell), hy = min((int)floorf((x.y + rr) * inv_cell), ly + 1);
    const int lz = (int)floorf((x.z - rr) * inv_cell), hz = min((int)floorf((x.z + rr) * inv_cell), lz + 1);
    uint32_t seen[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int cx = lx + (c & 1), cy = ly + ((c >> 1) & 1), cz = lz + ((c >> 2) & 1);
        const uint32_t h = cell_hash(cx, cy, cz, s, D.T);
        bool use = cx <= hx && cy <= hy && cz <= hz;
        seen[c] = use ? h : 0xFFFFFFFFu;
#pragma unroll
        for (int q = 0; q < c; ++q) use = use && seen[q] != h;
        if (!use) continue;
        const int e1 = D.start[h + 1];
        for (int e = D.start[h]; e < e1; ++e) {
            const float4 p = D.pts[e];
            const f3 dv = xyz(p) - x;
            const float d2 = dot3(dv, dv);
            if (!(d2 < R2) || fbits(p.w) != s) continue;
            ++m;
            if (mode == NEB_DENSITY_KNN) {
                float v = d2;
#pragma unroll
                for (int t = 0; t < kKnnMax; ++t) {
                    const float lo = fminf(best[t], v);
                    v = fmaxf(best[t], v);
                    best[t] = lo;
                }
            }
        }
    }
    if (mode == 0) return (float)m;
    if (mode == NEB_DENSITY_KNN && m >= k) {
        float dk = best[0];
#pragma unroll
        for (int t = 1; t < kKnnMax; ++t)
            if (t == k - 1) dk = best[t];
        return (float)k / (NEB_PI * dk);
    }
    return (float)m / (NEB_PI * R2);
}

// density of NEE vertices at x (geometric normal nn) in scene s, from the
// octree, the density grid or the analytic test density
__device__ __forceinline__ float point_density(const RenderArgs& A, int s, f3 x, f3 nn, const int32_t* __restrict__ nodes,
                                               const OctState* ost, const OctParams* prm, float scale) {
    if (A.density_mode == NEB_DENSITY_ANALYTIC) {
        const SceneInfo& I = A.sc[s];
        return I.rho0 + I.cam_w * cam_hit_density(I.cam, x, nn);
    }
    if (A.density_mode == NEB_DENSITY_RADIUS || A.density_mode == NEB_DENSITY_KNN) {
        const SceneInfo& I = A.sc[s];
        return set_density(A.dg, s, x, I.dr, I.inv_dcell, A.density_mode, I.knn_k);
    }
    if (A.density_mode == NEB_DENSITY_OCTREE) return oct_query(nodes, prm[s], scale, ost[s].depth, x, nn, false, nullptr);
    return oct_query_robust(nodes, prm[s], scale, ost[s].depth, x, nn);
}

// density grid over this iteration's NEE vertices: count -> scan -> scatter
// (count returns to zero after the scatter)
// (recycling = 1: the cells of the NEE recycling radius, and each entry's
// vertex index is kept)
__global__ void __launch_bounds__(256) k_dgrid_count(const SceneInfo* sc, VertexStore V, const int32_t* n_vertices,
                                                     DGrid D, int recycling) {
    const int n = *n_vertices;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int s = tag_scene(fbits(V.v1[i].w));
        const float inv = recycling ? sc[s].inv_ncell : sc[s].inv_dcell;
        atomicAdd(&D.count[point_hash(xyz(V.v0[i]), inv, s, D.T)], 1);
    }
}
__global__ void __launch_bounds__(256) k_dgrid_scatter(const SceneInfo* sc, VertexStore V, const int32_t* n_vertices,
                                                       DGrid D, int recycling) {
    const int n = *n_vertices;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int s = tag_scene(fbits(V.v1[i].w));
        const f3 p = xyz(V.v0[i]);
        const uint32_t h = point_hash(p, recycling ? sc[s].inv_ncell : sc[s].inv_dcell, s, D.T);
        const int pos = D.start[h] + atomicSub(&D.count[h], 1) - 1;
        D.pts[pos] = f4(p, ibits(s));
        if (recycling) D.vidx[pos] = i;
    }
}

// NEE recycling: n_E of every vertex, the NEE vertices within the radius
__global__ void __launch_bounds__(256) k_nee_count(RenderArgs A, VertexStore V, const int32_t* n_vertices) {
    const int n = *n_vertices;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int s = tag_scene(fbits(V.v1[i].w));
        const SceneInfo& I = A.sc[s];
        V.ne[i] = set_density(A.ng, s, xyz(V.v0[i]), I.nee_r, I.inv_ncell, 0, 1);
    }
}

// the same over a plain point set (neb_point_density; one scene, 0)
__global__ void __launch_bounds__(256) k_pset_count(const float* pts, int32_t n, float inv_cell, DGrid D) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        atomicAdd(&D.count[point_hash(mk3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]), inv_cell, 0, D.T)], 1);
}
__global__ void __launch_bounds__(256) k_pset_scatter(const float* pts, int32_t n, float inv_cell, DGrid D) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const f3 p = mk3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
        const uint32_t h = point_hash(p, inv_cell, 0, D.T);
        D.pts[D.start[h] + atomicSub(&D.count[h], 1) - 1] = f4(p, ibits(0));
    }
}
__global__ void __launch_bounds__(256) k_pset_query(const float* q, int32_t n, DGrid D, float R, float inv_cell, int mode,
                                                    int k, float* out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        out[i] = set_density(D, 0, mk3(q[3 * i], q[3 * i + 1], q[3 * i + 2]), R, inv_cell, mode, k);
}

__global__ void __launch_bounds__(256) k_density(RenderArgs A, VertexStore V, const int32_t* n_vertices,
                                                 const int32_t* __restrict__ nodes, const OctState* ost,
                                                 const OctParams* prm, const OctDyn* dyn) {
    int n = *n_vertices;
    const float scale = dyn->density_scale;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float4 a1 = V.v1[i];
        V.rho[i] = point_density(A, tag_scene(fbits(a1.w)), xyz(V.v0[i]), xyz(a1), nodes, ost, prm, scale);
    }
}

// ---------------------------------------------------------------------------
// pass 2 (b, c): NEE and the photon that reuses its segment
// ---------------------------------------------------------------------------
struct LightSample {
    f3 x, n, w, dE;
    float d2, cos_l, p_light;
    bool hittable;
    int lid;  // light pool index
};

// lights of one scene: [base, base + count) of the light pool, selected by
// the scene's cumulative power table: the first entry whose cdf exceeds u.
// The search starts at the guide entry of u's bucket floor(u count), the
// first light that the smallest uniform of the bucket can pick (so never
// past the answer), and steps forward: one or two table reads instead of a
// binary search's chain of dependent ones.  The bucket is taken from u's
// 24-bit grid value in integers, exactly.
__device__ __forceinline__ int pick_light(const SceneView& S, int base, int count, float u) {
    const uint32_t m = (uint32_t)(u * 16777216.0f);
    int i = S.light_guide[base + (int)(((uint64_t)m * (uint32_t)count) >> 24)];
    const float* cdf = S.light_cdf + base;
    while (i < count - 1 && !(u < cdf[i])) ++i;
    return base + i;
}

// Light pool entry (5 float4): l0 (p0 or position, selection probability),
// l1 (edge 1, area; 0 for a point light), l2 (edge 2), l3 (radiance or
// intensity), l4 (normal).  Emission density toward a receiver at squared
// distance d2 whose cosine is cx, in area measure at the receiver: cosine
// lobe cos_l / pi of an area light, 1 / (4 pi) of a point light.
__device__ __forceinline__ float emission_density(bool area, float cos_l, float cx, float d2) {
    return (area ? fmaxf(cos_l, 0.f) * (1.0f / NEB_PI) : 1.0f / (4.0f * NEB_PI)) * cx / d2;
}

__device__ __forceinline__ LightSample sample_light(const SceneView& S, int base, int count, f3 x, f3 nx,
                                                    const U4& u) {
    LightSample ls;
    ls.dE = mk3(0.f, 0.f, 0.f);
    ls.hittable = false;
    ls.p_light = 0.f;
    ls.cos_l = 0.f;
    ls.lid = pick_light(S, base, count, u.u[0]);
    const float4* L = S.lights + 5 * (size_t)ls.lid;
    float4 l0 = L[0], l1 = L[1], l2 = L[2], l3 = L[3];
    float psel = l0.w;
    if (l1.w > 0.f) {  // emissive triangle
        float su = sqrtf(u.u[1]);
        float b1 = u.u[2] * su;
        float b2 = 1.0f - (1.0f - su) - b1;
        f3 y = xyz(l0) + xyz(l1) * b1 + xyz(l2) * b2;
        f3 dv = y - x;
        float d2 = dot3(dv, dv);
        f3 w = dv * rsqrtf(d2);
        f3 ln = xyz(L[4]);
        ls.x = y;
        ls.n = ln;
        ls.w = w;
        ls.d2 = d2;
        ls.p_light = psel / l1.w;
        ls.hittable = true;
        float cl = -dot3(ln, w), cx = fabsf(dot3(nx, w));
        ls.cos_l = cl;
        if (cl > 0.f && cx > 0.f) ls.dE = xyz(l3) * (cx * cl / (d2 * ls.p_light));
    } else {  // point light: l3 holds the intensity
        f3 y = xyz(l0);
        f3 dv = y - x;
        float d2 = dot3(dv, dv);
        f3 w = dv * rsqrtf(d2);
        ls.x = y;
        ls.n = -w;
        ls.w = w;
        ls.d2 = d2;
        ls.p_light = psel;
        ls.cos_l = 1.f;
        float cx = fabsf(dot3(nx, w));
        if (cx > 0.f) ls.dE = xyz(l3) * (cx / (d2 * psel));
    }
    return ls;
}

// NEE (Sec. 3.1) in three launches over the vertices: k_nee_rays draws each
// vertex's light sample and queues a shadow ray where the sample carries
// energy (slots reserved once per block of 512 threads); a closest-hit launch in
// any-hit mode traces the queue (a lane takes the next ray when its own
// ends, so vertices without a ray leave no lane idle during traversal);
// k_nee_finish draws the same sample again (same stream), adds L_E and emits
// the NEB photon of every visible vertex.
constexpr int kNeeBlock = 512;
__global__ void __launch_bounds__(kNeeBlock) k_nee_rays(RenderArgs A, VertexStore V, const int32_t* n_vertices,
                                                        float4* __restrict__ s0, float4* __restrict__ s1,
                                                        float* __restrict__ stmax, int32_t* n_shadow) {
    __shared__ int wc[kNeeBlock / 64];
    __shared__ int bb;
    const int n = *n_vertices;
    const SceneView& S = A.S;
    const int iter = A.cnt->iter;
    for (int base = blockIdx.x * kNeeBlock; base < n; base += gridDim.x * kNeeBlock) {
        const int i = base + threadIdx.x;
        bool ray = false;
        f3 so = mk3(0.f, 0.f, 0.f), dir = so;
        float tmax = 0.f;
        int sid = 0;
        if (i < n) {
            float4 a0 = V.v0[i], a1 = V.v1[i];
            f3 x = xyz(a0), nrm = xyz(a1);
            int pixel = fbits(a0.w), tg = fbits(a1.w);
            int k = tag_depth(tg);
            sid = tag_scene(tg);
            const SceneInfo& I = A.sc[sid];
            U4 u = uniforms(I.k0, I.k1, (uint32_t)(pixel - I.pix_base), (uint32_t)iter, (uint32_t)k, kTagNee);
            LightSample ls = sample_light(S, I.light_base, I.n_lights, x, nrm, u);
            ray = !is_zero3(ls.dE);
            if (ray) {
                so = offset_origin(x, nrm, ls.w, I.eps);
                // An area light's sample point, rounded to floats, can sit a
                // few ulps behind its triangle; a grazing shadow ray would then
                // cross the emitter before its end.  The ray aims at the point
                // moved a tenth of the scene epsilon to the emitting side: a
                // convex emitter lies wholly behind that plane, and no other
                // surface comes that close to a light.
                f3 tgt = ls.hittable ? ls.x + ls.n * (0.1f * I.eps) : ls.x;
                f3 sd = tgt - so;
                float sl = sqrtf(dot3(sd, sd));
                dir = sd * (1.0f / sl);
                tmax = (1.0f - 1e-5f) * sl;
            }
        }
        const int slot = block_reserve<kNeeBlock / 64>(n_shadow, ray, wc, &bb);
        if (ray) {
            s0[slot] = f4(so, ibits(i));
            s1[slot] = f4(dir, ibits(make_tag(0, sid)));
            stmax[slot] = tmax;
        }
    }
}

// vis[i]: 1 if vertex i's shadow ray reached the light (read only where the
// sample carries energy, i.e. where k_nee_rays queued a ray)
__global__ void __launch_bounds__(kNeeBlock) k_nee_finish(RenderArgs A, VertexStore V, const int32_t* n_vertices,
                                                          const int32_t* __restrict__ visible, Images img,
                                                          PhotonQ pq, int32_t* pcount) {
    __shared__ int wc[kNeeBlock / 64];
    __shared__ int bb;
    const int n = *n_vertices;
    const SceneView& S = A.S;
    Counters* cnt = A.cnt;
    const int iter = cnt->iter;
    unsigned vis = 0, emitted = 0;
    for (int base = blockIdx.x * kNeeBlock; base < n; base += gridDim.x * kNeeBlock) {
        const int i = base + threadIdx.x;
        const bool valid = i < n;
        bool photon = false;
        Sample s;
        s.ev = 0;
        float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0, a2 = a0, a3 = a0;
        float rho = 0.f;
        if (valid) {
            a0 = V.v0[i];
            a1 = V.v1[i];
            a2 = V.v2[i];
            a3 = V.v3[i];
            rho = V.rho[i];
        }
        f3 x = xyz(a0), nrm = xyz(a1), wo = xyz(a2), tau = xyz(a3);
        int pixel = fbits(a0.w);
        int tg = fbits(a1.w);
        int k = tag_depth(tg), sid = tag_scene(tg), mid = tag_mat(tg);
        const SceneInfo& I = A.sc[sid];
        const uint32_t lpix = (uint32_t)(pixel - I.pix_base);
        const neb_material& m = S.mats[mid];
        LightSample ls;
        ls.dE = mk3(0.f, 0.f, 0.f);
        // light photons: emission density p_{l -> l-1} from the light point toward x
        float rem = 0.f;
        if (valid) {
            U4 u = uniforms(I.k0, I.k1, lpix, (uint32_t)iter, (uint32_t)k, kTagNee);
            ls = sample_light(S, I.light_base, I.n_lights, x, nrm, u);
            const bool ok = !is_zero3(ls.dE) && visible[i] != 0;
            // NEE recycling: the sample is kept for the neighbours, L_E comes later
            if (A.recycle) V.lsrec[i] = f4(ls.x, ibits(ok ? ls.lid : -1));
            if (ok) {
                ++vis;
                rem = emission_density(ls.hittable, ls.cos_l, fabsf(dot3(nrm, ls.w)), ls.d2);
                bool dnon = !mat_delta(m.type);
                if (dnon && !A.recycle) {
                    f3 f = bsdf_f(m, nrm, wo, ls.w);
                    if (!is_zero3(f)) {
                        float Am1 = (k >= 2) ? bsdf_pdf(m, nrm, ls.w, wo) * a3.w * a2.w : 0.f;
                        float ratio = 1.0f;
                        if (ls.hittable) ratio += bsdf_pdf(m, nrm, wo, ls.w) * ls.cos_l / (ls.d2 * ls.p_light);
                        if (A.photons) ratio += rho * I.r2pi * Am1;
                        ratio += I.nlp * I.r2pi * rem * (Am1 + 1.0f);
                        atomic_add3(img.E, pixel, tau * f * ls.dE * (1.0f / ratio));
                    }
                }
                if (A.photons && rho > 0.f) {
                    // the photon leaves the virtual light (counted), and enters
                    // the queue if its first scatter at x survives
                    ++emitted;
                    U4 up = uniforms(I.k0, I.k1, lpix, (uint32_t)iter, (uint32_t)(16 * k), kTagPhoton);
                    s = bsdf_sample(m, nrm, ls.w, up);
                    photon = s.ev != 0;
                }
            }
        }
        const int slot = block_reserve<kNeeBlock / 64>(pcount, photon, wc, &bb);
        if (photon) {
            float fo = ls.hittable ? bsdf_pdf(m, nrm, s.dir, ls.w) * ls.cos_l / (ls.d2 * ls.p_light) : 0.f;
            float dnon = mat_delta(m.type) ? 0.f : 1.f;
            // with light photons every merge of this photon gains the factor 1 + c
            // (c = n_LP p_{l -> l-1} / rho): folded into the flux and into U
            float c1 = 1.0f + I.nlp * rem / rho;
            // n_E NEE events at this vertex (NEE recycling), else 1
            const float ne = A.recycle ? V.ne[i] : 1.0f;
            float U1 = ((fo + dnon * ne) / (rho * I.r2pi) + (c1 - 1.0f) * dnon) / c1;
            float hp = fabsf(dot3(nrm, s.dir)) / s.pdf;
            f3 phi = ls.dE * (1.0f / (rho * c1)) * s.w;
            pq.p0[slot] = f4(offset_origin(x, nrm, s.dir, I.eps), ibits(pixel));
            pq.p1[slot] = f4(s.dir, ibits(make_tag(16 * k + 1, sid)));
            pq.p2[slot] = f4(phi, hp);
            pq.pu[slot] = U1;
        }
    }
    StatLine& L = stat_line(cnt);
    wave_add_u64(&L.nee_visible, vis);
    wave_add_u64(&L.photons, emitted);
}

// ---------------------------------------------------------------------------
// pass 2 (d): conventional light photons (Sec. 4, eq. stdphotonpdf)
// ---------------------------------------------------------------------------
// Light photon i of a scene picks a light by power and a point on it
// (stream LIGHT, word 0) and a direction (word 1): the cosine lobe around an
// area light's normal, the uniform sphere for a point light.  Its flux,
// L_e pi / p_light (area) or 4 pi I / P_sel (point), is shared by the n_LP
// photons.  The photons take the first entries of photon queue 0 (the NEB
// photons follow), tagged origin depth 0, bounce 0; until the first hit the
// U slot holds the light's pool index.
__global__ void __launch_bounds__(256) k_lp_emit(RenderArgs A, PhotonQ pq, int32_t* pcount) {
    const SceneView& S = A.S;
    Counters* cnt = A.cnt;
    const int iter = cnt->iter;
    unsigned emitted = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < A.n_lp; i += gridDim.x * blockDim.x) {
        const int sid = scene_of_pixel(A.lp_base, A.n_scenes, i);
        const SceneInfo& I = A.sc[sid];
        const int li = i - I.lp_base;
        bool go = scene_active(I, iter);
        f3 o = mk3(0.f, 0.f, 0.f), d = mk3(0.f, 0.f, 1.f), phi = o;
        int lid = 0;
        if (go) {
            U4 u = uniforms(I.k0, I.k1, (uint32_t)li, (uint32_t)iter, 0u, kTagLight);
            U4 v = uniforms(I.k0, I.k1, (uint32_t)li, (uint32_t)iter, 1u, kTagLight);
            lid = pick_light(S, I.light_base, I.n_lights, u.u[0]);
            const float4* L = S.lights + 5 * (size_t)lid;
            float4 l0 = L[0], l1 = L[1];
            f3 rad = xyz(L[3]);
            float sp, cp;
            sincosf(2.0f * NEB_PI * v.u[1], &sp, &cp);
            if (l1.w > 0.f) {  // emissive triangle
                float su = sqrtf(u.u[1]);
                float b1 = u.u[2] * su;
                float b2 = 1.0f - (1.0f - su) - b1;
                f3 y = xyz(l0) + xyz(l1) * b1 + xyz(L[2]) * b2;
                f3 ln = xyz(L[4]), t1, t2;
                basis(ln, t1, t2);
                float r = sqrtf(v.u[0]), z = sqrtf(fmaxf(0.f, 1.0f - v.u[0]));
                d = normalize3(t1 * (r * cp) + t2 * (r * sp) + ln * z);
                go = dot3(d, ln) > 0.f;
                phi = rad * (NEB_PI * l1.w / (l0.w * I.nlp));  // L_e pi / p_light, p_light = P_sel / area
                o = offset_origin(y, ln, d, I.eps);
            } else {  // point light: l3 holds the intensity
                float z = 1.0f - 2.0f * v.u[0], r = sqrtf(fmaxf(0.f, 1.0f - z * z));
                d = mk3(r * cp, r * sp, z);
                phi = rad * (4.0f * NEB_PI / (l0.w * I.nlp));
                o = xyz(l0);
            }
        }
        int slot = wave_reserve(pcount, go);
        wave_reserve(&cnt->lp_count, go);
        if (go) {
            ++emitted;
            pq.p0[slot] = f4(o, ibits(I.pix_base + li));
            pq.p1[slot] = f4(d, ibits(make_tag(0, sid)));
            pq.p2[slot] = f4(phi, 0.f);
            pq.pu[slot] = ibits(lid);
        }
    }
    wave_add_u64(&stat_line(cnt).light_photons, emitted);
}

// First hit y of each light photon (after the first closest-hit pass).  The
// paths these photons form have x_{l-1} = y; their NEB technique needs rho
// there, so it is queried here.  With p_{l -> l-1} the emission density
// toward y, n_LP p_{l -> l-1} sets the scale of the light-photon technique
// and c' = rho / (n_LP p_{l -> l-1}) that of the NEB photons relative to it.
// Every merge of the photon gains the factor 1 + c', which is folded into its
// flux; the merge at y itself has the MIS denominator
//   e + A_{k-1} + pdf_k(camera side -> light) X,
// with e = (1 + 1 / (n_LP pi r^2 p_{l -> l-1})) / (1 + c') and
// X = [area light] / (|cos at y| p_light n_LP r^2 (1 + c')), stored in p2.w
// and U for k_photon.  A photon whose emission density vanishes (grazing
// hit) carries no weight and is dropped.
__global__ void __launch_bounds__(256) k_lp_first(RenderArgs A, PhotonQ pq, int2* hits,
                                                  const int32_t* __restrict__ nodes, const OctState* ost,
                                                  const OctParams* prm, const OctDyn* dyn) {
    const int n = A.cnt->lp_count;
    const SceneView& S = A.S;
    const float scale = dyn->density_scale;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int2 h = hits[i];
        if (h.y < 0) continue;
        float4 b0 = pq.p0[i], b1 = pq.p1[i], b2 = pq.p2[i];
        const int sid = tag_scene(fbits(b1.w));
        const SceneInfo& I = A.sc[sid];
        f3 o = xyz(b0), d = xyz(b1);
        f3 y = o + d * ibits(h.x);
        f3 ny = xyz(S.prim_n[h.y]);
        const float4* L = S.lights + 5 * (size_t)fbits(pq.pu[i]);
        float4 l0 = L[0], l1 = L[1];
        const bool area = l1.w > 0.f;
        f3 ln = xyz(L[4]);
        f3 v = y - (area ? o - ln * I.eps : o);  // from the light point, before the ray offset
        float d2 = dot3(v, v);
        f3 w = v * rsqrtf(d2);
        float cos_y = fabsf(dot3(ny, w));
        float p_light = area ? l0.w / l1.w : l0.w;
        float rl = emission_density(area, dot3(ln, w), cos_y, d2);
        float rho = A.photons ? point_density(A, sid, y, ny, nodes, ost, prm, scale) : 0.f;
        float c1 = 1.0f + rho / (I.nlp * rl);
        float e = (1.0f + 1.0f / (I.nlp * I.r2pi * rl)) / c1;
        float X = area ? 1.0f / (cos_y * p_light * I.nlp * I.r * I.r * c1) : 0.f;
        if (!(rl > 0.f) || !isfinite(e) || !isfinite(X) || !isfinite(c1)) {
            hits[i] = make_int2(h.x, -1);
            continue;
        }
        pq.p2[i] = f4(xyz(b2) * (1.0f / c1), e);
        pq.pu[i] = X;
    }
}

// ---------------------------------------------------------------------------
// pass 2 (b'): NEE recycling (Sec. 6, the subsection on reusing NEE events)
// ---------------------------------------------------------------------------
// Every non-delta vertex evaluates the light samples of the n_E NEE vertices
// within the recycling radius (its own included) with its own BSDF: a light
// sample does not depend on the receiver, only the visibility tested by the
// vertex that drew it is borrowed.  With n_E samples of technique E the
// balance heuristic gives each sample c_j / (n_E + f_m / p_l + rho pi r^2 A).
__global__ void __launch_bounds__(256) k_nee_recycle(RenderArgs A, VertexStore V, const int32_t* n_vertices,
                                                     Images img) {
    const int n = *n_vertices;
    const SceneView& S = A.S;
    const DGrid& D = A.ng;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float4 a1 = V.v1[i];
        const int tg = fbits(a1.w);
        const neb_material& m = S.mats[tag_mat(tg)];
        if (mat_delta(m.type)) continue;
        const float4 a0 = V.v0[i], a2 = V.v2[i], a3 = V.v3[i];
        const int k = tag_depth(tg), s = tag_scene(tg);
        const SceneInfo& I = A.sc[s];
        const f3 x = xyz(a0), nrm = xyz(a1), wo = xyz(a2), tau = xyz(a3);
        const float rho = V.rho[i], ne = V.ne[i];
        const float R = I.nee_r, R2 = R * R, inv = I.inv_ncell, rr = R * 1.00001f;
        const int lx = (int)floorf((x.x - rr) * inv), hx = min((int)floorf((x.x + rr) * inv), lx + 1);
        const int ly = (int)floorf((x.y - rr) * inv), hy = min((int)floorf((x.y + rr) * inv), ly + 1);
        const int lz = (int)floorf((x.z - rr) * inv), hz = min((int)floorf((x.z + rr) * inv), lz + 1);
        f3 sum = mk3(0.f, 0.f, 0.f);
        uint32_t seen[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int cx = lx + (c & 1), cy = ly + ((c >> 1) & 1), cz = lz + ((c >> 2) & 1);
            const uint32_t h = cell_hash(cx, cy, cz, s, D.T);
            bool use = cx <= hx && cy <= hy && cz <= hz;
            seen[c] = use ? h : 0xFFFFFFFFu;
#pragma unroll
            for (int q = 0; q < c; ++q) use = use && seen[q] != h;
            if (!use) continue;
            const int e1 = D.start[h + 1];
            for (int e = D.start[h]; e < e1; ++e) {
                const float4 p = D.pts[e];
                const f3 dq = xyz(p) - x;
                if (!(dot3(dq, dq) < R2) || fbits(p.w) != s) continue;
                const float4 rec = V.lsrec[D.vidx[e]];
                const int lid = fbits(rec.w);
                if (lid < 0) continue;
                const float4* L = S.lights + 5 * (size_t)lid;
                const float4 l0 = L[0], l1 = L[1];
                const bool area = l1.w > 0.f;
                const f3 dv = xyz(rec) - x;
                const float d2 = dot3(dv, dv);
                const f3 w = dv * rsqrtf(d2);
                const float cx = fabsf(dot3(nrm, w));
                const float p_light = area ? l0.w / l1.w : l0.w;
                float cl = 1.f;
                if (area) cl = -dot3(xyz(L[4]), w);
                if (!(cl > 0.f) || !(cx > 0.f)) continue;
                const f3 dE = xyz(L[3]) * (cx * cl / (d2 * p_light));
                const f3 f = bsdf_f(m, nrm, wo, w);
                if (is_zero3(f)) continue;
                float den = ne;
                if (area) den += bsdf_pdf(m, nrm, wo, w) * cl / (d2 * p_light);
                if (A.photons && k >= 2) den += rho * I.r2pi * bsdf_pdf(m, nrm, w, wo) * a3.w * a2.w;
                sum = sum + tau * f * dE * (1.0f / den);
            }
        }
        if (!is_zero3(sum)) atomic_add3(img.E, fbits(a0.w), sum);
    }
}

// ---------------------------------------------------------------------------
// merge structure: hash grid of cell size 2r over the non-delta view vertices
// (count, which also gives each vertex its rank within its key -> exclusive
// scan, which zeroes the counts for the next iteration -> scatter to
// start[key] + rank)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t grid_key(const Grid& G, uint32_t h, int depth) {
    return (int64_t)h * G.D + (min(depth, G.D) - 1);
}

__global__ void __launch_bounds__(256) k_grid_count(const neb_material* mats, const SceneInfo* sc, VertexStore V,
                                                    const int32_t* n_vertices, Grid G) {
    int n = *n_vertices;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int tg = fbits(V.v1[i].w);
        if (mat_delta(mats[tag_mat(tg)].type)) continue;
        int s = tag_scene(tg);
        G.rank[i] = atomicAdd(&G.count[grid_key(G, point_hash(xyz(V.v0[i]), sc[s].inv_cell, s, G.T), tag_depth(tg))], 1);
    }
}

__global__ void __launch_bounds__(256) k_grid_scatter(const neb_material* mats, const SceneInfo* sc, VertexStore V,
                                                      const int32_t* n_vertices, Grid G) {
    int n = *n_vertices;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float4 a1 = V.v1[i];
        int tg = fbits(a1.w);
        if (mat_delta(mats[tag_mat(tg)].type)) continue;
        int s = tag_scene(tg);
        float4 a0 = V.v0[i];
        f3 p = xyz(a0);
        int64_t key = grid_key(G, point_hash(p, sc[s].inv_cell, s, G.T), tag_depth(tg));
        int pos = G.start[key] + G.rank[i];
        G.sorted[pos] = f4(p, ibits(s | (tag_depth(tg) << 24)));
        float4* m = G.mrec + 4 * (size_t)pos;
        m[0] = a1;
        m[1] = V.v2[i];
        m[2] = V.v3[i];
        m[3] = make_float4(a0.w, 0.f, 0.f, 0.f);
    }
}

// exclusive scan: 4096 elements per block of 256 threads

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wid; ++w) wbase += sh[w];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return wbase + x - v;
}

// zero_in: clear the input after reading it (in and out must not alias)
__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(int32_t* in, int32_t* out, int32_t* sums, int64_t n,
                                                           int zero_in) {
    __shared__ int sh[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int loc[kScanPer];
    int s = 0;
    if (base + kScanPer <= n && (((uintptr_t)(in + base)) & 15) == 0) {
        // a whole run of 16 ints, as four 16-byte loads
        const int4* v = reinterpret_cast<const int4*>(in + base);
#pragma unroll
        for (int k = 0; k < kScanPer / 4; ++k) {
            int4 w = v[k];
            loc[4 * k] = w.x;
            loc[4 * k + 1] = w.y;
            loc[4 * k + 2] = w.z;
            loc[4 * k + 3] = w.w;
        }
        if (zero_in) {
            int4* z = reinterpret_cast<int4*>(in + base);
#pragma unroll
            for (int k = 0; k < kScanPer / 4; ++k) z[k] = make_int4(0, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            loc[k] = (base + k < n) ? in[base + k] : 0;
            if (zero_in && base + k < n) in[base + k] = 0;
        }
    }
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += loc[k];
    int total;
    int pre = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int v = loc[k];
        loc[k] = pre;
        pre += v;
    }
    if (base + kScanPer <= n && (((uintptr_t)(out + base)) & 15) == 0) {
        int4* o = reinterpret_cast<int4*>(out + base);
#pragma unroll
        for (int k = 0; k < kScanPer / 4; ++k) o[k] = make_int4(loc[4 * k], loc[4 * k + 1], loc[4 * k + 2], loc[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k)
            if (base + k < n) out[base + k] = loc[k];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int32_t* sums, int32_t nb) {
    __shared__ int sh[4];
    int base = threadIdx.x * kScanPer;
    int loc[kScanPer];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        loc[k] = (base + k < nb) ? sums[base + k] : 0;
        s += loc[k];
    }
    int total;
    int pre = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < nb) sums[base + k] = pre;
        pre += loc[k];
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(int32_t* out, const int32_t* sums, int64_t n) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int add = sums[blockIdx.x];
    if (base + kScanPer <= n && (((uintptr_t)(out + base)) & 15) == 0) {
        int4* o = reinterpret_cast<int4*>(out + base);
#pragma unroll
        for (int k = 0; k < kScanPer / 4; ++k) {
            int4 w = o[k];
            o[k] = make_int4(w.x + add, w.y + add, w.z + add, w.w + add);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k)
            if (base + k < n) out[base + k] += add;
    }
}

// scratch ints needed by scan_exclusive for n elements (all levels)
static int64_t scan_scratch(int64_t n) {
    int64_t tot = 0;
    while (n > 1) {
        n = (n + kScanTile - 1) / kScanTile;
        tot += n;
    }
    return std::max<int64_t>(tot, 1);
}

// exclusive prefix sum of n ints (in and out may alias unless zero_in):
// tiles of 4096, then the tile sums recursively, then the offsets added
// back; zero_in clears the input as it is read
static void scan_exclusive(int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t s,
                           bool zero_in = false) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, scratch, n,
                       zero_in ? 1 : 0);
    if (nb <= kScanTile) {
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, scratch, (int32_t)nb);
    } else {
        scan_exclusive(scratch, scratch, nb, scratch + nb, s);
    }
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, out, scratch, n);
}

// photon order by bin (count -> exclusive scan -> this scatter); the bin
// counts return to zero
__global__ void __launch_bounds__(256) k_bin_scatter(const int32_t* __restrict__ bin, const int32_t* n_dev,
                                                     int32_t* count, const int32_t* __restrict__ start,
                                                     int32_t* __restrict__ order) {
    int n = *n_dev;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int b = bin[i];
        order[start[b] + atomicSub(&count[b], 1) - 1] = i;
    }
}

// ---------------------------------------------------------------------------
// photon bounce: merge with view vertices around the hit, then scatter.
// A wave takes 64 photons, one per lane; each lane finds the candidate
// ranges of its photon's cells.  The wave then walks the concatenation of
// all 64 photons' candidate lists together: consecutive lanes take
// consecutive candidates (a wave-wide scan of the lanes' counts maps a
// position back to its photon and cell), so the candidate loads of a step
// are contiguous runs of a cell's records and the number of steps follows
// the wave's total, not its longest list.  Accepted (photon, vertex) pairs
// are compacted into an LDS queue and evaluated 64 at a time by the whole
// wave, so the BSDF, the MIS weight and the image atomics run with every
// lane busy instead of with the ~15 % of candidates that are accepted.
// One wave per block.
// ---------------------------------------------------------------------------
// Photons are taken in the spatial order `order` (null: queue order).  Blocks
// b, b + 8, b + 16, ... run on one XCD (round-robin dispatch), so each XCD
// takes one contiguous eighth of the ordered photons: neighbouring photons
// then share that XCD's L2 for their cells and candidates.
// Four waves per SIMD (at most 128 VGPRs): with 10 000 bytes of LDS per
// block that is also the LDS limit, 16 resident blocks per CU.  Alone the
// kernel runs as fast with three; beside the closest hits and the camera
// pass the fourth keeps more of its loads in flight.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) k_photon(RenderArgs A, PhotonQ in, const int32_t* count_in, const int2* hits,
                                               Grid G, Images img, const int32_t* __restrict__ order) {
    __shared__ int2 queue[128];
    __shared__ float4 tp[64][2];  // per lane's photon: (-d, X), (Phi / (pi r^2), deepest mergeable depth | light bit)
    __shared__ float te[64];      // per lane's photon: weight of its own technique in the MIS denominator
    __shared__ float sval[64][3]; // contributions of a flushed batch
    __shared__ int sdst[64];      // their pixels (bit 30: light-photon image), -1 for none
    __shared__ int wbase[65];     // exclusive scan of the lanes' candidate counts
    __shared__ int coff[64][8];   // per lane's cell c: first record minus its offset in the lane's list
    __shared__ int cend[64][8];   // per lane's cell c: end of its range in the lane's list
    __shared__ float4 ty[64];     // per lane's photon: hit point, r^2
    __shared__ int tsid[64];      // per lane's photon: scene | deepest mergeable depth << 24
    const int lane = threadIdx.x;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int n = *count_in;
    const SceneView& S = A.S;
    Counters* cnt = A.cnt;
    const int iter = cnt->iter;
    unsigned segs = 0, merges = 0, items = 0, cells = 0, cands = 0;
    int qn = 0;  // queue length, identical in every lane

    // Evaluates up to 64 queued pairs, one per lane, then adds them to the
    // images with three lanes per pair (one colour channel each), so that the
    // three atomics of a pair go out in one instruction to one cache line.
    auto flush = [&](int count) {
        int dst = -1;
        f3 val = mk3(0.f, 0.f, 0.f);
        if (lane < count) {
            const int2 pr = queue[lane];
            // the whole 64-byte record at once (one line), so that the
            // material is the only load that waits for another
            const float4* mr = G.mrec + 4 * (size_t)pr.y;
            const float4 v1 = mr[0], v2 = mr[1], v3 = mr[2];
            const int pix = fbits(mr[3].x);
            const float4 t0 = tp[pr.x][0], t1 = tp[pr.x][1];
            const int tg = fbits(v1.w);
            const int k = tag_depth(tg);
            const int km = fbits(t1.w);
            if (k <= (km & 255)) {
                const neb_material& mv = S.mats[tag_mat(tg)];
                const f3 nv = xyz(v1), wv = xyz(v2), wd = xyz(t0);
                const f3 f = bsdf_f(mv, nv, wv, wd);
                if (!is_zero3(f)) {
                    const float T = bsdf_pdf(mv, nv, wv, wd) * t0.w;
                    const float C = te[pr.x] + ((k >= 2) ? bsdf_pdf(mv, nv, wd, wv) * v3.w * v2.w : 0.f);
                    dst = pix | ((km & 256) ? (1 << 30) : 0);
                    val = xyz(v3) * f * xyz(t1) * (1.0f / (C + T));
                    ++merges;
                }
            }
        }
        sdst[lane] = dst;
        sval[lane][0] = val.x;
        sval[lane][1] = val.y;
        sval[lane][2] = val.z;
        __syncthreads();
        const int sub = lane / 3, ch = lane - 3 * sub;
        for (int b = 0; b < count; b += 21) {
            const int m = b + sub;
            if (sub < 21 && m < count) {
                const int d = sdst[m];
                if (d >= 0)
                    atomicAdd(((d & (1 << 30)) ? img.LP : img.P) + 3 * (size_t)(d & ((1 << 30) - 1)) + ch, sval[m][ch]);
            }
        }
    };

    const int nchunk = (n + 63) >> 6;
    const int nblk = gridDim.x;
    int c_begin = blockIdx.x, c_end = nchunk, c_step = nblk;
    if (nblk >= 8) {
        const int x = blockIdx.x & 7, seg = (nchunk + 7) >> 3;
        c_begin = x * seg + (blockIdx.x >> 3);
        c_end = min(nchunk, (x + 1) * seg);
        c_step = (nblk - x + 7) >> 3;  // blocks on this XCD
    }
    for (int chunk = c_begin; chunk < c_end; chunk += c_step) {
        const int base = chunk * 64;
        int i = base + lane;
        bool valid = i < n;
        if (valid && order) i = order[i];
        int2 h = valid ? hits[i] : make_int2(0, -1);
        float4 b0 = make_float4(0.f, 0.f, 0.f, 0.f), b1 = b0, b2 = b0;
        float U = 0.f;
        if (valid) {
            b0 = in.p0[i];
            b1 = in.p1[i];
            b2 = in.p2[i];
            U = in.pu[i];
            ++items;
        }
        bool hit = h.y >= 0;
        int tg = fbits(b1.w);
        int code = tag_depth(tg), sid = tag_scene(tg);
        int j = code & 15, odepth = code >> 4, opix = fbits(b0.w);
        const SceneInfo& I = A.sc[sid];
        const float r = I.r, r2 = r * r, inv_cell = I.inv_cell, cell = 1.0f / inv_cell;
        f3 d = xyz(b1);
        f3 y = mk3(0.f, 0.f, 0.f), ny = mk3(0.f, 0.f, 1.f);
        float hh = 0.f;
        int mid = 0;
        if (hit) {
            ++segs;
            y = xyz(b0) + d * ibits(h.x);
            float4 pn = S.prim_n[h.y];
            ny = xyz(pn);
            mid = fbits(pn.w);
            hh = b2.w / fabsf(dot3(ny, d));
        }
        const neb_material& my = S.mats[mid];
        bool mergeable = hit && !mat_delta(my.type);
        // deepest view vertex this photon may merge with (a light photon's bounce
        // count is one less than its number of segments)
        const int kmax = I.L - 1 - j;
        // a light photon at its first hit brings the weight of its own technique
        // in p2.w and X in U; every other photon has weight 1 and X = h U
        const bool light = odepth == 0, lfirst = code == 0;
        const float X = lfirst ? U : hh * U, ef = lfirst ? b2.w : 1.0f;
        tp[lane][0] = f4(-d, X);
        tp[lane][1] = f4(xyz(b2) * (1.0f / I.r2pi), ibits(kmax | (light ? 256 : 0)));
        te[lane] = ef;
        // candidate ranges of the (at most 8) cells the ball touches.  The
        // lookups do not wait for the hit's material: a hit on a specular
        // surface (rare) drops its ranges afterwards
        int lo[8], pre[9];
        pre[0] = 0;
        unsigned looked = 0;
        {
            float rr = r * 1.00001f;
            int lx = (int)floorf((y.x - rr) * inv_cell), hx = min((int)floorf((y.x + rr) * inv_cell), lx + 1);
            int ly = (int)floorf((y.y - rr) * inv_cell), hy = min((int)floorf((y.y + rr) * inv_cell), ly + 1);
            int lz = (int)floorf((y.z - rr) * inv_cell), hz = min((int)floorf((y.z + rr) * inv_cell), lz + 1);
            uint32_t seen[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                int cx = lx + (c & 1), cy = ly + ((c >> 1) & 1), cz = lz + ((c >> 2) & 1);
                bool use = hit && kmax >= 1 && cx <= hx && cy <= hy && cz <= hz;
                // skip cells whose box is farther than r from the hit
                float dx = fmaxf(fmaxf(cx * cell - y.x, y.x - (cx + 1) * cell), 0.f);
                float dy = fmaxf(fmaxf(cy * cell - y.y, y.y - (cy + 1) * cell), 0.f);
                float dz = fmaxf(fmaxf(cz * cell - y.z, y.z - (cz + 1) * cell), 0.f);
                use = use && dx * dx + dy * dy + dz * dz <= r2 * 1.0001f;
                uint32_t hc = cell_hash(cx, cy, cz, sid, G.T);
                seen[c] = use ? hc : 0xFFFFFFFFu;
#pragma unroll
                for (int q = 0; q < c; ++q) use = use && seen[q] != hc;
                int e0 = 0, e1 = 0;
                if (use) {
                    int64_t key = grid_key(G, hc, 1);
                    e0 = G.start[key];
                    e1 = G.start[key + min(kmax, G.D)];
                    ++looked;
                }
                lo[c] = e0;
                pre[c + 1] = pre[c] + (e1 - e0);
            }
        }
        if (!mergeable) {
#pragma unroll
            for (int c = 1; c <= 8; ++c) pre[c] = 0;
            looked = 0;
        }
        cells += looked;
        int total = pre[8];
        cands += (unsigned)total;
        // the wave's candidate list: photon p's entries start at wbase[p];
        // its cell c covers [cend[p][c-1], cend[p][c]) of them, record
        // coff[p][c] + position
        int incl = total;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        const int wsum = __shfl(incl, 63, 64);
        wbase[lane + 1] = incl;
        if (lane == 0) wbase[0] = 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            coff[lane][c] = lo[c] - pre[c];
            cend[lane][c] = pre[c + 1];
        }
        ty[lane] = f4(y, r2);
        tsid[lane] = sid | (max(kmax, 0) << 24);
        __syncthreads();
        // four positions per lane per step, their loads independent (measured
        // on the room alone: 4 and 8 equal, both 22 % faster than one photon's
        // list per lane with eight loads in flight; beside the other streams
        // four is 1 % faster, sixteen 25 % slower)
        constexpr int kU = 4;
        for (int t = 0; t < wsum; t += 64 * kU) {
            int ev[kU], pv[kU];
            float4 cd[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int kk = t + u * 64 + lane;
                int e = -1, p = 0;
                if (kk < wsum) {
                    // p: the last photon whose list starts at or before kk
#pragma unroll
                    for (int st = 32; st; st >>= 1)
                        if (wbase[p + st] <= kk) p += st;
                    const int rk = kk - wbase[p];
                    int c = 0;
#pragma unroll
                    for (int q = 0; q < 7; ++q) c += cend[p][q] <= rk;
                    e = coff[p][c] + rk;
                }
                ev[u] = e;
                pv[u] = p;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) cd[u] = ev[u] >= 0 ? G.sorted[ev[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                bool acc = false;
                if (ev[u] >= 0) {
                    const float4 yp = ty[pv[u]];
                    f3 dv = xyz(cd[u]) - xyz(yp);
                    // a bucket may also hold another scene's cell, and the
                    // last depth class deeper vertices than the photon may reach
                    const int w = fbits(cd[u].w), ts = tsid[pv[u]];
                    acc = dot3(dv, dv) < yp.w && (w & 0xFFFFFF) == (ts & 0xFFFFFF) && (w >> 24) <= (ts >> 24);
                }
                unsigned long long m = __ballot(acc);
                if (m) {
                    if (acc) queue[qn + __popcll(m & below)] = make_int2(pv[u], ev[u]);
                    qn += __popcll(m);
                    if (qn >= 64) {
                        __syncthreads();
                        flush(64);
                        __syncthreads();
                        int2 rest = lane < qn - 64 ? queue[64 + lane] : make_int2(0, 0);
                        __syncthreads();
                        if (lane < qn - 64) queue[lane] = rest;
                        qn -= 64;
                        __syncthreads();
                    }
                }
            }
        }
        if (qn > 0) {
            __syncthreads();
            flush(qn);
            qn = 0;
        }
        __syncthreads();
    }
    StatLine& L = stat_line(cnt);
    wave_add_u64(&L.photon_segments, segs);
    wave_add_u64(&L.merges, merges);
    wave_add_u64(&L.photon_items, items);
    wave_add_u64(&L.grid_cells, cells);
    wave_add_u64(&L.candidates, cands);
}

// The scatter of a photon bounce (Sec. 3.2): every photon that hit a
// surface below its last bounce samples the BSDF there and continues; its
// factor U gains the term of the hit vertex.  A launch of its own, so that
// the merges of the bounce (k_photon, which reads the same queue and hits)
// can run beside the next bounce's closest-hit launch.  Slots are reserved
// once per block; count_copy receives the input count for the merge launch
// (the closest-hit launch that follows clears the count it read).
constexpr int kScatterBlock = 512;
__global__ void __launch_bounds__(kScatterBlock) k_pscatter(RenderArgs A, PhotonQ in, const int32_t* count_in,
                                                            const int2* __restrict__ hits, PhotonQ out,
                                                            int32_t* count_out, int32_t* count_copy) {
    __shared__ int wc[kScatterBlock / 64];
    __shared__ int bb;
    const int n = *count_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_copy = n;
    const SceneView& S = A.S;
    Counters* cnt = A.cnt;
    const int iter = cnt->iter;
    unsigned cont = 0;
    for (int base = blockIdx.x * kScatterBlock; base < n; base += gridDim.x * kScatterBlock) {
        const int i = base + threadIdx.x;
        bool go = false;
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
        float Un = 0.f;
        const int2 h = i < n ? hits[i] : make_int2(0, -1);
        if (h.y >= 0) {
            const float4 b0 = in.p0[i], b1 = in.p1[i], b2 = in.p2[i];
            const float U = in.pu[i];
            const int tg = fbits(b1.w);
            const int code = tag_depth(tg), sid = tag_scene(tg);
            const int j = code & 15, odepth = code >> 4, opix = fbits(b0.w);
            const SceneInfo& I = A.sc[sid];
            const f3 d = xyz(b1);
            const f3 y = xyz(b0) + d * ibits(h.x);
            const float4 pn = S.prim_n[h.y];
            const f3 ny = xyz(pn);
            const neb_material& my = S.mats[fbits(pn.w)];
            if (j < I.L - 2 && !mat_black(my)) {
                // a light photon at its first hit brings the weight of its own
                // technique in p2.w and X in U; every other photon has weight 1
                // and X = h U
                const bool lfirst = code == 0;
                const float hh = b2.w / fabsf(dot3(ny, d));
                const float X = lfirst ? U : hh * U, ef = lfirst ? b2.w : 1.0f;
                U4 u = uniforms(I.k0, I.k1, (uint32_t)(opix - I.pix_base), (uint32_t)iter, (uint32_t)(16 * odepth + j),
                                kTagPhoton);
                Sample s = bsdf_sample(my, ny, -d, u);
                go = s.ev != 0;
                if (go) {
                    const float prev = bsdf_pdf(my, ny, s.dir, -d);
                    Un = (mat_delta(my.type) ? 0.f : ef) + prev * X;
                    const float hp = fabsf(dot3(ny, s.dir)) / s.pdf;
                    r0 = f4(offset_origin(y, ny, s.dir, I.eps), ibits(opix));
                    r1 = f4(s.dir, ibits(make_tag(16 * odepth + j + 1, sid)));
                    r2 = f4(xyz(b2) * s.w, hp);
                }
            }
        }
        const int slot = block_reserve<kScatterBlock / 64>(count_out, go, wc, &bb);
        if (go) {
            ++cont;
            out.p0[slot] = r0;
            out.p1[slot] = r1;
            out.p2[slot] = r2;
            out.pu[slot] = Un;
        }
    }
    wave_add_u64(&stat_line(cnt).photon_continued, cont);
}

// ---------------------------------------------------------------------------
// pass 3: emitter hits
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_finalize(RenderArgs A, const float4* ev0, const float4* ev1,
                                                  const int32_t* n_events, const float* rho, const float* ne,
                                                  Images img) {
    int n = *n_events;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float4 a = ev0[i], b = ev1[i];
        float w = 1.0f;
        if (a.w > 0.f) {
            int pv = fbits(b.z);
            float ratio = b.y * (ne ? ne[pv] : 1.0f);  // n_E at x_{l-1} (NEE recycling)
            if (A.photons) ratio += rho[pv] * b.x;
            w = 1.0f / (1.0f + a.w * ratio);
        }
        atomic_add3(img.e, fbits(b.w), xyz(a) * w);
    }
}

// ---------------------------------------------------------------------------
// learned density: training pool, probes against the octree, region gates
// and the octree fallback (one scene per context)
// ---------------------------------------------------------------------------
constexpr int kRegionRes = 32;  // regions of the octree box per axis (octree depth 5)
constexpr int kRegions = kRegionRes * kRegionRes * kRegionRes;
enum {
    kMlpCntProbes = 0,
    kMlpCntBad = 1,
    kMlpCntFallback = 2,
    kMlpCntDisabled = 3,
    kMlpCntProbed = 4,
    kMlpCntServed = 5,     // probes so far in regions that keep the model
    kMlpCntServedBad = 6,  // ... of them over the bound
    kMlpCnt = 8
};

__device__ __forceinline__ int region_of(const OctParams& P, f3 p) {
    float v[3] = {p.x, p.y, p.z};
    int r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float q = __fmul_rn(__fsub_rn(v[c], P.min_bound[c]), P.size_inv[c]);
        r[c] = min(kRegionRes - 1, max(0, (int)(q * (float)kRegionRes)));
    }
    return r[0] + kRegionRes * (r[1] + kRegionRes * r[2]);
}

// the vertices with rho > 0 become the pool: position, normal, log rho
__global__ void __launch_bounds__(256) k_mlp_collect(VertexStore V, const int32_t* n_vertices, float* pos, float* nrm,
                                                     float* tgt, int32_t* count) {
    int n = *n_vertices;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float rho = V.rho[i];
        bool take = rho > 0.f;
        int slot = wave_reserve(count, take);
        if (take) {
            float4 a = V.v0[i], b = V.v1[i];
            pos[3 * (size_t)slot] = a.x;
            pos[3 * (size_t)slot + 1] = a.y;
            pos[3 * (size_t)slot + 2] = a.z;
            nrm[3 * (size_t)slot] = b.x;
            nrm[3 * (size_t)slot + 1] = b.y;
            nrm[3 * (size_t)slot + 2] = b.z;
            tgt[slot] = logf(rho);
        }
    }
}

// Compares the model's density (already in V.rho) with the robust octree
// query at every vertex (all != 0) or at a random subset, and adds the
// comparisons to the per-region tallies.  A vertex of the subset is picked
// by its own draw (pixel, iteration, depth; probe stream): with n vertices it
// is probed when its 24-bit uniform u satisfies u * n < n_probe * 2^24, so
// the expected number of probes is n_probe and the choice does not depend on
// the order of the vertex store.
__global__ void __launch_bounds__(256) k_mlp_probe(VertexStore V, const int32_t* n_vertices,
                                                   const int32_t* __restrict__ nodes, const OctState* ost,
                                                   OctParams P, const OctDyn* dyn, int all, int n_probe, uint32_t k0,
                                                   uint32_t k1, const Counters* cnt, int32_t* total, int32_t* bad,
                                                   float* sums, float max_rel, unsigned long long* mc) {
    const int nv = *n_vertices;
    const int depth = ost->depth;
    const float scale = dyn->density_scale;
    const uint32_t it = (uint32_t)cnt->iter;
    const uint64_t lim = (uint64_t)n_probe << 24;
    unsigned probes = 0, nbad = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
        float4 a0 = V.v0[i], a1 = V.v1[i];
        if (!all) {
            uint32_t x = philox10(make_uint4((uint32_t)fbits(a0.w), it, (uint32_t)tag_depth(fbits(a1.w)), kTagProbe),
                                  k0, k1).x;
            if ((uint64_t)(x >> 8) * (uint64_t)nv >= lim) continue;
        }
        f3 x = xyz(a0), nn = xyz(a1);
        float rm = V.rho[i];
        float ro = oct_query_robust(nodes, P, scale, depth, x, nn);
        bool b = ro > 0.f ? fabsf(rm - ro) > max_rel * ro : rm > 0.f;
        int r = region_of(P, x);
        atomicAdd(total + r, 1);
        if (b) atomicAdd(bad + r, 1);
        atomicAdd(sums + r, rm);
        atomicAdd(sums + kRegions + r, ro);
        ++probes;
        nbad += b;
    }
    wave_add_u64(mc + kMlpCntProbes, probes);
    wave_add_u64(mc + kMlpCntBad, nbad);
}

// A region keeps the model while the model's densities summed over the
// region's probes so far are within the bound of the octree's summed over
// the same probes: the model's bias there, relative.  (Probe by probe the
// octree's own counting noise -- a leaf of c deposits, c of the order of the
// split threshold, is a Poisson count -- is larger than a 10 % bound, so a
// per-probe rule would also reject an exact model; summed over a region's
// probes it averages out.)  A region without probes keeps the model.  Also
// tallies the probes of the regions that keep the model, and how many of
// those exceed the bound one by one.
__global__ void k_mlp_gate(const int32_t* total, const int32_t* bad, const float* sums, float max_rel, int32_t* gate,
                           unsigned long long* mc) {
    unsigned off = 0, probed = 0, served = 0, served_bad = 0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < kRegions; r += gridDim.x * blockDim.x) {
        const int t = total[r], b = bad[r];
        const float sm = sums[r], so = sums[kRegions + r];
        const bool on = t == 0 || (so > 0.f ? fabsf(sm - so) <= max_rel * so : !(sm > 0.f));
        gate[r] = on ? 1 : 0;
        off += !on;
        probed += t > 0;
        if (on) {
            served += t;
            served_bad += b;
        }
    }
    wave_add_u64(mc + kMlpCntDisabled, off);
    wave_add_u64(mc + kMlpCntProbed, probed);
    wave_add_u64(mc + kMlpCntServed, served);
    wave_add_u64(mc + kMlpCntServedBad, served_bad);
}

__global__ void k_mlp_clear_gate_counts(unsigned long long* mc) {
    mc[kMlpCntDisabled] = 0;
    mc[kMlpCntProbed] = 0;
    mc[kMlpCntServed] = 0;
    mc[kMlpCntServedBad] = 0;
}

// vertices in disabled regions take the robust octree query instead
__global__ void __launch_bounds__(256) k_density_fallback(VertexStore V, const int32_t* n_vertices,
                                                          const int32_t* __restrict__ gate,
                                                          const int32_t* __restrict__ nodes, const OctState* ost,
                                                          OctParams P, const OctDyn* dyn, unsigned long long* mc) {
    const int n = *n_vertices;
    const int depth = ost->depth;
    const float scale = dyn->density_scale;
    unsigned fb = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        f3 x = xyz(V.v0[i]);
        if (gate[region_of(P, x)]) continue;
        V.rho[i] = oct_query_robust(nodes, P, scale, depth, x, xyz(V.v1[i]));
        ++fb;
    }
    wave_add_u64(mc + kMlpCntFallback, fb);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int grid_of(int64_t n, int block, int cap = 8192) {
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace neb

using namespace neb;

static thread_local std::string g_err;

static neb_status fail(neb_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(NEB_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

struct neb_octree_s {
    Octree o;
};

// validated host copy of one scene of the batch
struct HostScene {
    bool set = false;
    BvhHost bvh;
    int32_t nt = 0;
    std::vector<float> prim_n;        // 4 per prim: unit normal, w = scene-local material id bits
    std::vector<int32_t> prim_light;  // scene-local light id or -1
    std::vector<float> lights;        // 20 floats per light
    std::vector<float> cdf;           // cumulative selection probabilities
    std::vector<neb_material> mats;
    float bmin[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
    CamParams cam{};
    float eps = 0.f;
};

// launch shapes picked by neb_autotune (or set by the caller)
// (defaults: the shapes the autotuner picks for the room workload; the
// stack is raised to the shallowest that holds the deepest tree)
struct LaunchCfg {
    int stack = 32;        // LDS traversal stack entries per lane: 32, 48 or 64
    int trace_bpc = 8;     // closest-hit blocks (one wave each) per CU; 0 = one block per 64 queue slots,
                           // -1 = as many as the LDS holds (clamped to that for deeper stacks)
    int nee_bpc = 16;      // NEE (shadow-ray) blocks per CU, same conventions
    int photon_bpc = 24;   // photon-merge blocks (one wave each) per CU; 0 = one block per 256 queue slots
    int photon_order = 0;  // merge photons in the spatial order of their hits
    int concurrent = 1;    // second stream for the work that can run beside other work
};

struct neb_ctx_s {
    int n_scenes = 0;
    std::vector<neb_params> prm;
    std::vector<HostScene> hs;
    std::vector<int32_t> pix_base;  // n_scenes + 1
    std::vector<int32_t> lp_base;   // n_scenes + 1: light photons per iteration of the scenes before
    int npix = 0, L = 0, n_lp = 0;
    int64_t vcap = 0, ecap = 0, slot_cap = 0;
    int64_t pcap = 0;               // photon queue entries: NEB photons (<= vertices) + light photons
    int density_mode = 0, flags = 0, photons = 1;
    int cus = 256;
    // per-scene device tables and the shared geometry pools
    bool ready = false;  // forest uploaded and octrees initialised since the last scene change
    int forest_depth = 0;  // traversal stack entries the forest's deepest descent needs
    SceneInfo* sc_dev = nullptr;
    int32_t* pix_base_dev = nullptr;
    int32_t* lp_base_dev = nullptr;
    std::vector<SceneInfo> sc_host;
    SceneView view{};
    std::vector<void*> scene_allocs;
    // octree pool: scene s owns [oct_prm[s].root, oct_prm[s].end)
    int32_t* oct_nodes = nullptr;
    OctState* oct_states = nullptr;
    OctParams* oct_prm_dev = nullptr;
    OctDyn* oct_dyn = nullptr;
    std::vector<OctParams> oct_prm;
    int64_t oct_total = 0;
    int32_t* defer[2] = {nullptr, nullptr};
    int32_t* defer_cnt = nullptr;
    // per-iteration pools
    PathQ q[2]{};
    PhotonQ pq[kPhotonBufs]{};
    // a second stream (default priority) for NEE's shadow rays, the
    // merge-grid build and the merges, forked after shading; joined before
    // NEE's contributions (ev_nee), before a bounce's scatter overwrites the
    // queue that the merges two bounces back read, and at the end of the
    // bounces (ev_merge[j]: the merges of bounce j).  A third stream (cam,
    // below) runs the next iteration's camera pass.
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_nee = nullptr;
    hipEvent_t ev_merge[kMaxPathLen + 1]{};
    int2* phits[kPhotonBufs]{};  // hit arrays of the photon queues (the first is hits)
    float4 *sq0 = nullptr, *sq1 = nullptr;  // NEE shadow rays: (origin, vertex), (direction, tag)
    float* sqt = nullptr;                   // their tmax
    int32_t* svis = nullptr;                // per vertex: 1 if its shadow ray reached the light
    int2* hits = nullptr;
    // Two vertex and event stores, by the parity of the iteration: the
    // camera pass of the next iteration (on a third stream, cam) fills one
    // while this iteration's photon bounces and pass 3 read the other.  V,
    // ev0, ev1, nvtx and nevt are the current iteration's.
    VertexStore Vb[2]{};
    float4 *ev0b[2]{}, *ev1b[2]{};
    VertexStore V{};
    float4 *ev0 = nullptr, *ev1 = nullptr;
    int32_t *nvtx = nullptr, *nevt = nullptr;
    int2* chits = nullptr;  // closest hits of the camera pass
    hipStream_t cam = nullptr;
    hipEvent_t ev_cam_fork = nullptr, ev_cam_done = nullptr;
    int32_t* slots = nullptr;
    neb_path_record* recs = nullptr;
    Grid G{};
    DGrid dg{};  // NEB_DENSITY_RADIUS / NEB_DENSITY_KNN
    DGrid ng{};  // NEE recycling
    int recycle = 0;
    // spatial order of photon hits
    int32_t *pbin = nullptr, *porder = nullptr, *bcount = nullptr, *bstart = nullptr, *bsums = nullptr;
    int32_t bin_bits = 0, n_bins = 0;
    float* img = nullptr;  // e, E, P, LP accumulators, 3 * npix floats each
    Counters* cnt = nullptr;
    int32_t iter = 0;
    int32_t first_iter_recorded = 0;
    hipStream_t last_stream = nullptr;
    std::vector<void*> allocs;
    LaunchCfg cfg;
    // captured iterations, by (parity, camera pass inline, next camera pass forked)
    int use_graph = 0;  // 1: one graph per iteration, 2: one graph per call
    hipGraph_t graph[8]{};
    hipGraphExec_t gexec[8]{};
    // captured calls (use_graph 2), by their iteration count
    static constexpr int kCallGraphs = 4;
    int32_t call_n[kCallGraphs]{};
    hipGraph_t call_graph[kCallGraphs]{};
    hipGraphExec_t call_exec[kCallGraphs]{};
    int call_next = 0;  // slot the next capture replaces
    hipStream_t cap_stream = nullptr;
    // learned density (NEB_DENSITY_MLP)
    bool mlp_mode = false;
    neb_mlp_params mcfg{};
    Mlp mlp;
    // a model given by neb_set_mlp_model: its parameters and normalisation
    // replace the seeded initial weights and the first pool's statistics
    bool mlp_given = false;
    std::vector<float> mlp_init;
    float mlp_mu = 0.f, mlp_sigma = 1.f;
    float *tpos = nullptr, *tnrm = nullptr, *ttgt = nullptr;  // training pool
    int32_t* tcount = nullptr;
    int32_t *reg_total = nullptr, *reg_bad = nullptr, *reg_gate = nullptr;
    float* reg_sum = nullptr;  // per region: model and octree densities summed over its probes (2 x kRegions)
    unsigned long long* mlp_cnt = nullptr;
    int32_t last_train_steps = 0;
    // kernel profiling
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_kid;
    int prof_used = 0;
    double prof_ms[32] = {0};
    int64_t prof_launches[32] = {0};
};

enum KernelId {
    K_CAMERA, K_EXTEND_CAMERA, K_SHADE, K_OCTREE_INSERT, K_DENSITY, K_NEE, K_GRID_BUILD, K_EXTEND_PHOTON, K_PHOTON,
    K_FINALIZE, K_MLP_TRAIN, K_PHOTON_ORDER, K_MISC, K_LIGHT_PHOTON, K_DENSITY_GRID, K_NEE_RECYCLE, K_PHOTON_SCATTER,
    K_COUNT
};
static const char* kKernelNames[K_COUNT] = {"camera", "extend_camera", "shade", "octree_insert", "density", "nee",
                                            "grid_build", "extend_photon", "photon_merge", "finalize", "mlp_train",
                                            "photon_order", "misc", "light_photon", "density_grid", "nee_recycle",
                                            "photon_scatter"};

static void prof_harvest(neb_ctx c) {
    if (c->prof_used == 0) return;
    for (int i = 0; i < c->prof_used; i += 2) {
        float ms = 0.f;
        // the pairs sit on up to three streams: wait for each
        (void)hipEventSynchronize(c->prof_ev[i + 1]);
        if (hipEventElapsedTime(&ms, c->prof_ev[i], c->prof_ev[i + 1]) == hipSuccess) {
            c->prof_ms[c->prof_kid[i / 2]] += ms;
            c->prof_launches[c->prof_kid[i / 2]] += 1;
        }
    }
    c->prof_used = 0;
}

static void prof_clear(neb_ctx c) {
    prof_harvest(c);
    for (int k = 0; k < 32; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_launches[k] = 0;
    }
}

static hipError_t prof_alloc(neb_ctx c) {
    if (!c->prof_ev.empty()) return hipSuccess;
    c->prof_ev.resize(4096);
    c->prof_kid.resize(2048);
    for (auto& e : c->prof_ev) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

static void prof_begin(neb_ctx c, int kid, hipStream_t s) {
    if (!c->prof_on) return;
    if (c->prof_used + 2 > (int)c->prof_ev.size()) prof_harvest(c);
    c->prof_kid[c->prof_used / 2] = kid;
    (void)hipEventRecord(c->prof_ev[c->prof_used], s);
}

static void prof_end(neb_ctx c, hipStream_t s) {
    if (!c->prof_on) return;
    (void)hipEventRecord(c->prof_ev[c->prof_used + 1], s);
    c->prof_used += 2;
}

#define TIMED(kid, ...)          \
    do {                         \
        prof_begin(c, (kid), s); \
        __VA_ARGS__;             \
        prof_end(c, s);          \
    } while (0)

template <typename T>
static hipError_t dalloc(std::vector<void*>& list, T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(1, count) * sizeof(T));
    if (e == hipSuccess) {
        list.push_back(q);
        *p = (T*)q;
    }
    return e;
}

static void free_list(std::vector<void*>& l) {
    for (void* p : l) (void)hipFree(p);
    l.clear();
}

static neb_status oom_or_device(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return fail(NEB_ERR_OUT_OF_MEMORY, std::string("out of device memory: ") + what);
    return fail(NEB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

extern "C" const char* neb_status_string(neb_status s) {
    switch (s) {
    case NEB_OK: return "ok";
    case NEB_ERR_INVALID_ARG: return "invalid argument";
    case NEB_ERR_OUT_OF_MEMORY: return "out of memory";
    case NEB_ERR_CAPACITY: return "capacity exceeded";
    case NEB_ERR_DEVICE: return "device error";
    case NEB_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

extern "C" const char* neb_last_error(void) { return g_err.c_str(); }

static uint32_t next_pow2(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return (uint32_t)p;
}

static int lds_blocks_per_cu(int stack) { return (160 * 1024) / (stack * kTraceBlock * 4); }

// blocks of a traversal launch over a queue of at most cap rays, with bpc
// blocks per CU (0: one block per 64 queue slots, -1: as many as the LDS holds)
static int trace_grid(neb_ctx c, int64_t cap, int bpc) {
    if (bpc < 0 || bpc > lds_blocks_per_cu(c->cfg.stack)) bpc = lds_blocks_per_cu(c->cfg.stack);
    // never more blocks than the queue has lanes' worth of rays: a small
    // queue would leave most blocks without work
    if (bpc > 0) return std::max(1, (int)std::min<int64_t>((int64_t)c->cus * bpc, (cap + kTraceBlock - 1) / kTraceBlock));
    return grid_of(cap, kTraceBlock, 1 << 20);
}

static void drop_graph(neb_ctx c) {
    for (int k = 0; k < 8; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
        c->gexec[k] = nullptr;
        c->graph[k] = nullptr;
    }
    for (int k = 0; k < neb_ctx_s::kCallGraphs; ++k) {
        if (c->call_exec[k]) (void)hipGraphExecDestroy(c->call_exec[k]);
        if (c->call_graph[k]) (void)hipGraphDestroy(c->call_graph[k]);
        c->call_exec[k] = nullptr;
        c->call_graph[k] = nullptr;
        c->call_n[k] = 0;
    }
    c->call_next = 0;
}

static void destroy_ctx(neb_ctx c) {
    drop_graph(c);
    mlp_free(c->mlp);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->cam) (void)hipStreamDestroy(c->cam);
    if (c->ev_cam_fork) (void)hipEventDestroy(c->ev_cam_fork);
    if (c->ev_cam_done) (void)hipEventDestroy(c->ev_cam_done);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_nee) (void)hipEventDestroy(c->ev_nee);
    for (auto& e : c->ev_merge)
        if (e) (void)hipEventDestroy(e);
    free_list(c->scene_allocs);
    free_list(c->allocs);
    for (auto& e : c->prof_ev) (void)hipEventDestroy(e);
    delete c;
}

static void mlp_defaults(neb_mlp_params& m) {
    m.train_iterations = 4;
    m.steps_per_iteration = 250;
    m.batch = 65536;
    m.lr = 2e-3f;
    m.beta1 = 0.9f;
    m.beta2 = 0.999f;
    m.eps = 1e-8f;
    m.probe_every = 8;
    m.probes = 4096;
    m.max_rel_error = 0.1f;
    m.seed = 1;
}

// He-uniform weights (bound sqrt(6 / fan_in)) and zero biases
static std::vector<float> mlp_he_init(uint32_t seed) {
    std::vector<float> w(kMlpParams, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int n, int fan_in) {
        std::uniform_real_distribution<double> u(-std::sqrt(6.0 / fan_in), std::sqrt(6.0 / fan_in));
        for (int i = 0; i < n; ++i) w[off + i] = (float)u(rng);
    };
    fill(kMlpW1, kMlpIn * kMlpWidth, kMlpIn);
    fill(kMlpW2, kMlpWidth * kMlpWidth, kMlpWidth);
    fill(kMlpW3, kMlpWidth * kMlpWidth, kMlpWidth);
    fill(kMlpW4, kMlpWidth, kMlpWidth);
    return w;
}

static neb_status check_params(const neb_params* p) {
    if (p->width < 1 || p->height < 1 || p->width > 8192 || p->height > 8192)
        return fail(NEB_ERR_INVALID_ARG, "image size out of range");
    if (p->max_path_len < 1 || p->max_path_len > kMaxPathLen) return fail(NEB_ERR_INVALID_ARG, "max_path_len out of range");
    if (p->octree_capacity < 1 || p->octree_capacity > (1 << 29)) return fail(NEB_ERR_INVALID_ARG, "octree capacity out of range");
    if (!(p->merge_radius > 0.f) || !std::isfinite(p->merge_radius)) return fail(NEB_ERR_INVALID_ARG, "merge radius must be > 0");
    if (p->density_mode != NEB_DENSITY_OCTREE && p->density_mode != NEB_DENSITY_OCTREE_ROBUST &&
        p->density_mode != NEB_DENSITY_ANALYTIC && p->density_mode != NEB_DENSITY_MLP &&
        p->density_mode != NEB_DENSITY_RADIUS && p->density_mode != NEB_DENSITY_KNN)
        return fail(NEB_ERR_INVALID_ARG, "unknown density mode");
    if (p->density_mode == NEB_DENSITY_RADIUS || p->density_mode == NEB_DENSITY_KNN) {
        if (!(p->density_radius > 0.f) || !std::isfinite(p->density_radius))
            return fail(NEB_ERR_INVALID_ARG, "density_radius must be > 0");
        if (p->density_mode == NEB_DENSITY_KNN && (p->knn_k < 1 || p->knn_k > kKnnMax))
            return fail(NEB_ERR_INVALID_ARG, "knn_k out of range (1 .. 16)");
    }
    if (!std::isfinite(p->analytic_rho0) || !std::isfinite(p->analytic_cam_weight))
        return fail(NEB_ERR_INVALID_ARG, "analytic density parameters must be finite");
    if (p->spp < 0) return fail(NEB_ERR_INVALID_ARG, "spp must be >= 0");
    if (p->light_photons < 0 || p->light_photons > (1 << 26))
        return fail(NEB_ERR_INVALID_ARG, "light_photons out of range (0 .. 2^26)");
    if (!(p->nee_radius >= 0.f) || !std::isfinite(p->nee_radius))
        return fail(NEB_ERR_INVALID_ARG, "nee_radius must be >= 0");
    if (p->nee_radius > 0.f && p->light_photons > 0)
        return fail(NEB_ERR_INVALID_ARG, "NEE recycling is not combined with light photons");
    return NEB_OK;
}

extern "C" neb_status neb_create_batch(const neb_params* params, int32_t n_scenes, neb_ctx* out) {
    if (!params || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    if (n_scenes < 1 || n_scenes > kMaxScenes) return fail(NEB_ERR_INVALID_ARG, "scene count out of range (1..256)");
    int64_t npix = 0, vcap = 0, ecap = 0, oct_total = 0, n_lp = 0;
    int L = 0;
    for (int s = 0; s < n_scenes; ++s) {
        neb_status st = check_params(params + s);
        if (st != NEB_OK) return st;
        const neb_params& p = params[s];
        if (p.density_mode != params[0].density_mode || p.flags != params[0].flags)
            return fail(NEB_ERR_INVALID_ARG, "every scene of a batch needs the same density mode and flags");
        if ((p.nee_radius > 0.f) != (params[0].nee_radius > 0.f))
            return fail(NEB_ERR_INVALID_ARG, "NEE recycling must be on for every scene of a batch or for none");
        int64_t np = (int64_t)p.width * p.height;
        npix += np;
        vcap += np * std::max(1, p.max_path_len - 1);
        ecap += np * p.max_path_len;
        oct_total += octree_capacity_rounded(p.octree_capacity);
        L = std::max(L, p.max_path_len);
        n_lp += p.max_path_len >= 2 ? p.light_photons : 0;
    }
    if (npix > (int64_t)INT32_MAX / 16 || vcap * 4 > (int64_t)INT32_MAX || ecap > (int64_t)INT32_MAX)
        return fail(NEB_ERR_CAPACITY, "images too large for the vertex pool");
    if (oct_total >= (int64_t)INT32_MAX - 16) return fail(NEB_ERR_CAPACITY, "octree pool over 2^31 nodes");
    if (params[0].density_mode == NEB_DENSITY_MLP && n_scenes != 1)
        return fail(NEB_ERR_INVALID_ARG, "the learned density needs a context of one scene");
    if (params[0].density_mode == NEB_DENSITY_MLP && n_lp > 0)
        return fail(NEB_ERR_INVALID_ARG, "light photons need the octree or the analytic density");
    if (vcap + n_lp > (int64_t)INT32_MAX / 4) return fail(NEB_ERR_CAPACITY, "too many photons per iteration");
    int64_t slot_cap = npix * std::max(1, L - 1);
    if ((params[0].flags & NEB_FLAG_SINGLE_THREAD_OCTREE) && slot_cap > (int64_t)INT32_MAX)
        return fail(NEB_ERR_CAPACITY, "too many pixels for single-thread deposits");

    neb_ctx c = new neb_ctx_s();
    c->n_scenes = n_scenes;
    c->prm.assign(params, params + n_scenes);
    c->hs.resize(n_scenes);
    c->pix_base.resize(n_scenes + 1);
    c->lp_base.resize(n_scenes + 1);
    c->oct_prm.resize(n_scenes);
    c->sc_host.resize(n_scenes);
    {
        int64_t pb = 0, root = 0, lb = 0;
        for (int s = 0; s < n_scenes; ++s) {
            c->pix_base[s] = (int32_t)pb;
            pb += (int64_t)params[s].width * params[s].height;
            c->lp_base[s] = (int32_t)lb;
            lb += params[s].max_path_len >= 2 ? params[s].light_photons : 0;
            OctParams& P = c->oct_prm[s];
            std::memset(&P, 0, sizeof(P));
            P.root = (int32_t)root;
            P.end = (int32_t)(root + octree_capacity_rounded(params[s].octree_capacity));
            root = P.end;
        }
        c->pix_base[n_scenes] = (int32_t)pb;
        c->lp_base[n_scenes] = (int32_t)lb;
    }
    c->n_lp = (int)n_lp;
    c->pcap = vcap + n_lp;
    c->npix = (int)npix;
    c->L = L;
    c->vcap = vcap;
    c->ecap = ecap;
    c->slot_cap = slot_cap;
    c->oct_total = oct_total;
    c->density_mode = params[0].density_mode;
    c->flags = params[0].flags;
    c->photons = (c->flags & NEB_FLAG_NO_PHOTONS) ? 0 : 1;
    c->recycle = params[0].nee_radius > 0.f ? 1 : 0;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            c->cus = cus;
    }
    hipError_t e = hipSuccess;
#define ALLOC(ptr, n)                                   \
    if (e == hipSuccess) e = dalloc(c->allocs, &(ptr), (size_t)(n));
    for (int b = 0; b < 2; ++b) {
        ALLOC(c->q[b].q0, npix);
        ALLOC(c->q[b].q1, npix);
        ALLOC(c->q[b].q2, npix);
        ALLOC(c->q[b].q3, npix);
    }
    for (int b = 0; b < kPhotonBufs; ++b) {
        ALLOC(c->pq[b].p0, c->pcap);
        ALLOC(c->pq[b].p1, c->pcap);
        ALLOC(c->pq[b].p2, c->pcap);
        ALLOC(c->pq[b].pu, c->pcap);
    }
    ALLOC(c->hits, c->pcap);
    ALLOC(c->chits, npix);
    c->phits[0] = c->hits;
    for (int b = 1; b < kPhotonBufs; ++b) ALLOC(c->phits[b], c->pcap);
    ALLOC(c->sq0, vcap);
    ALLOC(c->sq1, vcap);
    ALLOC(c->sqt, vcap);
    ALLOC(c->svis, vcap);
    for (int b = 0; b < 2; ++b) {
        ALLOC(c->Vb[b].v0, vcap);
        ALLOC(c->Vb[b].v1, vcap);
        ALLOC(c->Vb[b].v2, vcap);
        ALLOC(c->Vb[b].v3, vcap);
        ALLOC(c->Vb[b].rho, vcap);
        ALLOC(c->ev0b[b], ecap);
        ALLOC(c->ev1b[b], ecap);
    }
    if (c->flags & NEB_FLAG_SINGLE_THREAD_OCTREE) ALLOC(c->slots, slot_cap);
    if (c->flags & NEB_FLAG_RECORD_PATHS) ALLOC(c->recs, npix * L);
    // eight depth classes whatever the path length: a cell's row is one
    // aligned 32-byte sector, and the table's size does not grow with the
    // path length (longer paths share the last class)
    c->G.D = 8;
    c->G.T = (int32_t)std::max<uint64_t>(1024, std::min<uint64_t>(next_pow2((uint64_t)vcap) / 2, 1u << 23));
    int64_t gkeys = (int64_t)c->G.T * c->G.D + 1;
    ALLOC(c->G.count, gkeys);
    ALLOC(c->G.start, gkeys);
    ALLOC(c->G.rank, vcap);
    ALLOC(c->G.sorted, vcap);
    ALLOC(c->G.mrec, 4 * vcap);
    ALLOC(c->G.sums, scan_scratch(gkeys));
    if (c->recycle) {
        c->ng.T = c->G.T;
        ALLOC(c->ng.count, (int64_t)c->ng.T + 1);
        ALLOC(c->ng.start, (int64_t)c->ng.T + 1);
        ALLOC(c->ng.pts, vcap);
        ALLOC(c->ng.vidx, vcap);
        ALLOC(c->ng.sums, scan_scratch((int64_t)c->ng.T + 1));
        for (int b = 0; b < 2; ++b) {
            ALLOC(c->Vb[b].ne, vcap);
            ALLOC(c->Vb[b].lsrec, vcap);
        }
    }
    if (c->density_mode == NEB_DENSITY_RADIUS || c->density_mode == NEB_DENSITY_KNN) {
        c->dg.T = c->G.T;
        ALLOC(c->dg.count, (int64_t)c->dg.T + 1);
        ALLOC(c->dg.start, (int64_t)c->dg.T + 1);
        ALLOC(c->dg.pts, vcap);
        ALLOC(c->dg.sums, scan_scratch((int64_t)c->dg.T + 1));
    }
    ALLOC(c->img, 12 * npix);
    ALLOC(c->cnt, 1);
    ALLOC(c->oct_nodes, oct_total);
    ALLOC(c->oct_states, n_scenes);
    ALLOC(c->oct_prm_dev, n_scenes);
    ALLOC(c->oct_dyn, 1);
    ALLOC(c->defer[0], vcap);
    ALLOC(c->defer[1], vcap);
    ALLOC(c->defer_cnt, 3);
    ALLOC(c->sc_dev, n_scenes);
    ALLOC(c->pix_base_dev, n_scenes + 1);
    ALLOC(c->lp_base_dev, n_scenes + 1);
    {
        // about 2^18 bins over all scenes, 2..6 bits per axis
        int bits = 6;
        while (bits > 2 && ((int64_t)n_scenes << (3 * bits)) > (1 << 18)) --bits;
        c->bin_bits = bits;
        c->n_bins = n_scenes << (3 * bits);
    }
    ALLOC(c->pbin, c->pcap);
    ALLOC(c->porder, c->pcap);
    ALLOC(c->bcount, c->n_bins + 2);
    ALLOC(c->bstart, c->n_bins + 2);
    ALLOC(c->bsums, scan_scratch(c->n_bins + 2));
    if (c->density_mode == NEB_DENSITY_MLP) {
        c->mlp_mode = true;
        mlp_defaults(c->mcfg);
        ALLOC(c->tpos, 3 * vcap);
        ALLOC(c->tnrm, 3 * vcap);
        ALLOC(c->ttgt, vcap);
        ALLOC(c->tcount, 1);
        ALLOC(c->reg_total, kRegions);
        ALLOC(c->reg_bad, kRegions);
        ALLOC(c->reg_gate, kRegions);
        ALLOC(c->reg_sum, 2 * kRegions);
        ALLOC(c->mlp_cnt, kMlpCnt);
        if (e == hipSuccess) e = mlp_alloc(c->mlp, c->mcfg.batch);
    }
#undef ALLOC
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(gkeys, 256)), dim3(256), 0, nullptr, c->G.count, 0, gkeys);
        if (c->dg.count)
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_of((int64_t)c->dg.T + 1, 256)), dim3(256), 0, nullptr, c->dg.count,
                               0, (int64_t)c->dg.T + 1);
        if (c->ng.count)
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_of((int64_t)c->ng.T + 1, 256)), dim3(256), 0, nullptr, c->ng.count,
                               0, (int64_t)c->ng.T + 1);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(c->n_bins + 2, 256)), dim3(256), 0, nullptr, c->bcount, 0,
                           (int64_t)c->n_bins + 2);
        hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(12 * npix, 256)), dim3(256), 0, nullptr, c->img, 0.f, 12 * npix);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, nullptr, (int32_t*)c->cnt, 0,
                           (int64_t)(sizeof(Counters) / 4));
        e = hipMemcpy(c->pix_base_dev, c->pix_base.data(), 4 * c->pix_base.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(c->lp_base_dev, c->lp_base.data(), 4 * c->lp_base.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        neb_status s = oom_or_device(e, "neb_create");
        destroy_ctx(c);
        return s;
    }
    *out = c;
    return NEB_OK;
}

extern "C" neb_status neb_create(const neb_params* p, neb_ctx* out) { return neb_create_batch(p, 1, out); }

static bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// validates one scene and builds its BVH and light table on the host
static neb_status build_host_scene(const neb_params& prm, const float* vertices, int32_t nv, const int32_t* tris,
                                   const int32_t* tri_material, int32_t nt, const neb_material* materials, int32_t nm,
                                   const neb_point_light* point_lights, int32_t npl, const neb_camera* camera,
                                   HostScene& H) {
    if (!vertices || !tris || !tri_material || !materials || !camera) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (nv < 3 || nt < 1 || nm < 1 || npl < 0 || (npl > 0 && !point_lights))
        return fail(NEB_ERR_INVALID_ARG, "bad scene sizes");
    if (nm > kMaxMaterials) return fail(NEB_ERR_CAPACITY, "more than 65536 materials");
    float bmin[3] = {INFINITY, INFINITY, INFINITY}, bmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < nv; ++i) {
        if (!finite3(vertices + 3 * i)) return fail(NEB_ERR_INVALID_ARG, "non-finite vertex");
        for (int k = 0; k < 3; ++k) {
            bmin[k] = std::min(bmin[k], vertices[3 * i + k]);
            bmax[k] = std::max(bmax[k], vertices[3 * i + k]);
        }
    }
    for (int k = 0; k < 3; ++k)
        if (!(bmax[k] > bmin[k])) return fail(NEB_ERR_INVALID_ARG, "flat scene bounding box");
    for (int64_t t = 0; t < nt; ++t) {
        for (int k = 0; k < 3; ++k)
            if (tris[3 * t + k] < 0 || tris[3 * t + k] >= nv) return fail(NEB_ERR_INVALID_ARG, "triangle index out of range");
        if (tri_material[t] < 0 || tri_material[t] >= nm) return fail(NEB_ERR_INVALID_ARG, "material index out of range");
    }
    for (int i = 0; i < nm; ++i) {
        const neb_material& m = materials[i];
        if (m.type < 0 || m.type > 3) return fail(NEB_ERR_INVALID_ARG, "unknown material type");
        if (!finite3(m.albedo) || !finite3(m.emission) || !std::isfinite(m.ior) || !std::isfinite(m.alpha))
            return fail(NEB_ERR_INVALID_ARG, "non-finite material");
        if (m.type == NEB_MAT_DIELECTRIC && !(m.ior > 0.f)) return fail(NEB_ERR_INVALID_ARG, "ior must be > 0");
        if (m.type == NEB_MAT_GGX && !(m.alpha > 0.f)) return fail(NEB_ERR_INVALID_ARG, "GGX alpha must be > 0");
    }
    for (int i = 0; i < npl; ++i)
        if (!finite3(point_lights[i].pos) || !finite3(point_lights[i].power))
            return fail(NEB_ERR_INVALID_ARG, "non-finite point light");
    if (!finite3(camera->eye) || !finite3(camera->look_at) || !finite3(camera->up) ||
        !(camera->vfov_deg > 0.f && camera->vfov_deg < 180.f))
        return fail(NEB_ERR_INVALID_ARG, "bad camera");
    // camera basis
    CamParams& C = H.cam;
    double f[3], up[3], r[3], u[3];
    for (int k = 0; k < 3; ++k) {
        C.eye[k] = camera->eye[k];
        f[k] = (double)camera->look_at[k] - camera->eye[k];
        up[k] = camera->up[k];
    }
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0)) return fail(NEB_ERR_INVALID_ARG, "camera looks at its own position");
    for (double& x : f) x /= fl;
    r[0] = f[1] * up[2] - f[2] * up[1];
    r[1] = f[2] * up[0] - f[0] * up[2];
    r[2] = f[0] * up[1] - f[1] * up[0];
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 0)) return fail(NEB_ERR_INVALID_ARG, "camera up is parallel to the view direction");
    for (double& x : r) x /= rl;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    for (int k = 0; k < 3; ++k) {
        C.f[k] = (float)f[k];
        C.r[k] = (float)r[k];
        C.u[k] = (float)u[k];
    }
    C.tan_half = (float)std::tan(0.5 * camera->vfov_deg * M_PI / 180.0);
    C.aspect = (float)prm.width / (float)prm.height;
    C.w = prm.width;
    C.h = prm.height;

    // BVH
    if (!build_bvh(vertices, nv, tris, nt, H.bvh)) return fail(NEB_ERR_INVALID_ARG, "BVH build failed");
    if (H.bvh.stack_need >= kBvhStackMax) return fail(NEB_ERR_CAPACITY, "BVH needs a deeper traversal stack");
    // per-prim normals and light table (emissive triangles, then point lights)
    H.nt = nt;
    H.prim_n.assign(4 * (size_t)nt, 0.f);
    H.prim_light.assign(nt, -1);
    H.lights.clear();
    std::vector<double> w;
    auto emis = [&](const neb_material& m) { return ((double)m.emission[0] + m.emission[1] + m.emission[2]) / 3.0; };
    for (int64_t t = 0; t < nt; ++t) {
        const float* a = vertices + 3 * (size_t)tris[3 * t];
        const float* b = vertices + 3 * (size_t)tris[3 * t + 1];
        const float* cc = vertices + 3 * (size_t)tris[3 * t + 2];
        double e1[3], e2[3], cr[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = (double)b[k] - a[k];
            e2[k] = (double)cc[k] - a[k];
        }
        cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
        cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
        cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        for (int k = 0; k < 3; ++k) H.prim_n[4 * t + k] = len > 0 ? (float)(cr[k] / len) : (k == 2 ? 1.f : 0.f);
        int32_t mid = tri_material[t];
        std::memcpy(&H.prim_n[4 * t + 3], &mid, 4);
        const neb_material& m = materials[mid];
        if (emis(m) > 0.0 && len > 0) {
            H.prim_light[t] = (int32_t)w.size();
            double area = 0.5 * len;
            w.push_back(M_PI * area * emis(m));
            float L0[20] = {a[0], a[1], a[2], 0.f,
                            (float)e1[0], (float)e1[1], (float)e1[2], (float)area,
                            (float)e2[0], (float)e2[1], (float)e2[2], 0.f,
                            m.emission[0], m.emission[1], m.emission[2], 0.f,
                            H.prim_n[4 * t], H.prim_n[4 * t + 1], H.prim_n[4 * t + 2], 0.f};
            H.lights.insert(H.lights.end(), L0, L0 + 20);
        }
    }
    for (int i = 0; i < npl; ++i) {
        const neb_point_light& l = point_lights[i];
        w.push_back(((double)l.power[0] + l.power[1] + l.power[2]) / 3.0);
        const double inv4pi = 1.0 / (4.0 * M_PI);
        float L0[20] = {l.pos[0], l.pos[1], l.pos[2], 0.f,
                        0.f, 0.f, 0.f, 0.f,
                        0.f, 0.f, 0.f, 1.f,
                        (float)(l.power[0] * inv4pi), (float)(l.power[1] * inv4pi), (float)(l.power[2] * inv4pi), 0.f,
                        0.f, 0.f, 0.f, 0.f};
        H.lights.insert(H.lights.end(), L0, L0 + 20);
    }
    int nl = (int)w.size();
    if (nl == 0) return fail(NEB_ERR_INVALID_ARG, "scene has no lights");
    double tot = 0.0;
    for (double x : w) tot += x;
    if (!(tot > 0.0)) return fail(NEB_ERR_INVALID_ARG, "scene lights carry no power");
    // Uniforms are multiples of 2^-24, so u < c holds exactly when u is below
    // c rounded up to that grid; the grid values are exact floats, and the
    // device's float comparison then picks the light the exact cumulative
    // sum picks (rounding c to the nearest float would move a boundary
    // across a grid point now and then).
    H.cdf.assign(nl, 0.f);
    double acc = 0.0;
    for (int i = 0; i < nl; ++i) {
        acc += w[i];
        H.cdf[i] = (float)(std::ceil(acc / tot * 16777216.0) / 16777216.0);
        H.lights[20 * (size_t)i + 3] = (float)(w[i] / tot);
    }
    H.cdf[nl - 1] = 1.0f;
    H.mats.assign(materials, materials + nm);
    for (int k = 0; k < 3; ++k) {
        H.bmin[k] = bmin[k];
        H.bmax[k] = bmax[k];
    }
    float dg[3] = {bmax[0] - bmin[0], bmax[1] - bmin[1], bmax[2] - bmin[2]};
    H.eps = 1e-5f * std::sqrt(dg[0] * dg[0] + dg[1] * dg[1] + dg[2] * dg[2]);
    H.set = true;
    return NEB_OK;
}

// clears images, counters and every octree of the batch; iteration 0
static neb_status restart(neb_ctx c, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(12 * (int64_t)c->npix, 256)), dim3(256), 0, s, c->img, 0.f,
                       12 * (int64_t)c->npix);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int32_t*)c->cnt, 0, (int64_t)(sizeof(Counters) / 4));
    for (int i = 0; i < c->n_scenes; ++i)
        HIP_TRY(octree_init_range(c->oct_nodes, c->oct_states + i, c->oct_prm[i].root,
                                  c->oct_prm[i].end - c->oct_prm[i].root, s));
    OctDyn d0;
    octree_dyn_for(d0, 1);
    HIP_TRY(octree_set_dyn(c->oct_dyn, d0, s));
    if (c->mlp_mode) {
        std::vector<float> w = c->mlp_given ? c->mlp_init : mlp_he_init(c->mcfg.seed);
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(mlp_set_weights(c->mlp, w.data(), s));
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(mlp_set_norm(c->mlp, c->mlp_given ? c->mlp_mu : 0.f, c->mlp_given ? c->mlp_sigma : 1.f, s));
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(kRegions, 256)), dim3(256), 0, s, c->reg_total, 0, (int64_t)kRegions);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(kRegions, 256)), dim3(256), 0, s, c->reg_bad, 0, (int64_t)kRegions);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(kRegions, 256)), dim3(256), 0, s, c->reg_gate, 1, (int64_t)kRegions);
        hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(2 * kRegions, 256)), dim3(256), 0, s, c->reg_sum, 0.f,
                           (int64_t)(2 * kRegions));
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int32_t*)c->mlp_cnt, 0, (int64_t)(2 * kMlpCnt));
        c->last_train_steps = 0;
    }
    HIP_TRY(hipGetLastError());
    c->iter = 0;
    c->first_iter_recorded = 0;
    return NEB_OK;
}

// Concatenates the scenes into the shared pools (BVH forest with per-scene
// roots, triangles, prim tables, materials, lights), writes the per-scene
// tables and initialises the octrees.  Runs once after the scenes change.
static neb_status prepare(neb_ctx c) {
    if (c->ready) return NEB_OK;
    for (int s = 0; s < c->n_scenes; ++s)
        if (!c->hs[s].set) return fail(NEB_ERR_STATE, "scene " + std::to_string(s) + " not set");
    drop_graph(c);
    int64_t n_nodes = 0, n_tris = 0, n_mats = 0, n_lights = 0;
    int depth = 0;
    for (const HostScene& H : c->hs) {
        n_nodes += H.bvh.n_nodes;
        n_tris += H.nt;
        n_mats += (int64_t)H.mats.size();
        n_lights += (int64_t)H.cdf.size();
        depth = std::max(depth, H.bvh.stack_need);
    }
    if (n_mats > kMaxMaterials) return fail(NEB_ERR_CAPACITY, "more than 65536 materials over the batch");
    if (n_nodes * 8 > (int64_t)INT32_MAX || n_tris * 3 > (int64_t)INT32_MAX || n_lights * 5 > (int64_t)INT32_MAX)
        return fail(NEB_ERR_CAPACITY, "geometry pools over 2^31 entries");
    std::vector<float> nodes(32 * (size_t)n_nodes), tri(12 * (size_t)n_tris), prim_n(4 * (size_t)n_tris),
        lights(20 * (size_t)n_lights), cdf((size_t)n_lights);
    std::vector<int32_t> guide((size_t)n_lights);
    std::vector<int32_t> prim_light((size_t)n_tris);
    std::vector<neb_material> mats((size_t)n_mats);
    int64_t nb = 0, tb = 0, mb = 0, lb = 0;
    for (int s = 0; s < c->n_scenes; ++s) {
        const HostScene& H = c->hs[s];
        const neb_params& P = c->prm[s];
        // nodes: child links are node indices (inner) or triangle indices (leaves)
        for (int i = 0; i < H.bvh.n_nodes; ++i) {
            const float* src = &H.bvh.nodes[32 * (size_t)i];
            float* dst = &nodes[32 * (size_t)(nb + i)];
            std::memcpy(dst, src, 32 * 4);
            int32_t lk[4], ct[4];
            std::memcpy(lk, src + 24, 16);
            std::memcpy(ct, src + 28, 16);
            for (int ch = 0; ch < 4; ++ch) {
                if (ct[ch] > 0) lk[ch] += (int32_t)tb;
                else if (lk[ch] >= 0) lk[ch] += (int32_t)nb;
            }
            std::memcpy(dst + 24, lk, 16);
        }
        for (int t = 0; t < H.nt; ++t) {
            const float* src = &H.bvh.tris[12 * (size_t)t];
            float* dst = &tri[12 * (size_t)(tb + t)];
            std::memcpy(dst, src, 48);
            int32_t pid;
            std::memcpy(&pid, src + 3, 4);
            pid += (int32_t)tb;
            std::memcpy(dst + 3, &pid, 4);
            float* pn = &prim_n[4 * (size_t)(tb + t)];
            std::memcpy(pn, &H.prim_n[4 * (size_t)t], 16);
            int32_t mid;
            std::memcpy(&mid, pn + 3, 4);
            mid += (int32_t)mb;
            std::memcpy(pn + 3, &mid, 4);
            prim_light[tb + t] = H.prim_light[t] >= 0 ? H.prim_light[t] + (int32_t)lb : -1;
        }
        std::copy(H.mats.begin(), H.mats.end(), mats.begin() + mb);
        std::copy(H.lights.begin(), H.lights.end(), lights.begin() + 20 * lb);
        std::copy(H.cdf.begin(), H.cdf.end(), cdf.begin() + lb);
        {
            // guide entry k: the first light whose cumulative value (c / 2^24,
            // c an integer: the table lies on the uniforms' grid) exceeds the
            // smallest uniform m_min / 2^24 of bucket k, m_min = ceil(k 2^24 / n)
            const int n = (int)H.cdf.size();
            int i = 0;
            for (int k = 0; k < n; ++k) {
                const uint64_t m_min = (((uint64_t)k << 24) + (uint64_t)n - 1) / (uint64_t)n;
                while (i < n - 1 && (uint64_t)std::llround((double)H.cdf[i] * 16777216.0) <= m_min) ++i;
                guide[lb + k] = i;
            }
        }
        SceneInfo& I = c->sc_host[s];
        std::memset(&I, 0, sizeof(I));
        I.cam = H.cam;
        I.pix_base = c->pix_base[s];
        I.npix = P.width * P.height;
        I.L = P.max_path_len;
        I.spp = P.spp;
        I.bvh_root = (int32_t)nb;
        I.light_base = (int32_t)lb;
        I.n_lights = (int32_t)H.cdf.size();
        I.k0 = P.seed;
        I.k1 = P.scene_id;
        I.eps = H.eps;
        I.r = P.merge_radius;
        I.r2pi = (float)(M_PI * (double)P.merge_radius * (double)P.merge_radius);
        I.inv_cell = 1.0f / (2.0001f * P.merge_radius);  // a little wider than the ball's diameter
        I.rho0 = P.analytic_rho0;
        I.cam_w = P.analytic_cam_weight;
        I.n_lp = P.max_path_len >= 2 ? P.light_photons : 0;
        I.lp_base = c->lp_base[s];
        I.nlp = (float)I.n_lp;
        I.dr = P.density_radius;
        I.inv_dcell = P.density_radius > 0.f ? 1.0f / (2.0001f * P.density_radius) : 0.f;
        I.knn_k = P.knn_k;
        I.nee_r = P.nee_radius;
        I.inv_ncell = P.nee_radius > 0.f ? 1.0f / (2.0001f * P.nee_radius) : 0.f;
        OctParams& O = c->oct_prm[s];
        octree_params_init(O, H.bmin, H.bmax, O.root, P.octree_capacity);
        nb += H.bvh.n_nodes;
        tb += H.nt;
        mb += (int64_t)H.mats.size();
        lb += (int64_t)H.cdf.size();
    }
    free_list(c->scene_allocs);
    float4 *d_nodes = nullptr, *d_tri = nullptr, *d_pn = nullptr, *d_lights = nullptr;
    int32_t* d_pl = nullptr;
    float* d_cdf = nullptr;
    int32_t* d_guide = nullptr;
    neb_material* d_mats = nullptr;
    hipError_t e = dalloc(c->scene_allocs, &d_nodes, 8 * (size_t)n_nodes);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &d_tri, 3 * (size_t)n_tris);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &d_pn, (size_t)n_tris);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &d_pl, (size_t)n_tris);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &d_mats, (size_t)n_mats);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &d_lights, 5 * (size_t)n_lights);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &d_cdf, (size_t)n_lights);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &d_guide, (size_t)n_lights);
    if (e != hipSuccess) return oom_or_device(e, "scene upload");
    HIP_TRY(hipMemcpy(d_nodes, nodes.data(), nodes.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_tri, tri.data(), tri.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_pn, prim_n.data(), prim_n.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_pl, prim_light.data(), prim_light.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_mats, mats.data(), mats.size() * sizeof(neb_material), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_lights, lights.data(), lights.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_cdf, cdf.data(), cdf.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_guide, guide.data(), guide.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->sc_dev, c->sc_host.data(), sizeof(SceneInfo) * c->sc_host.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->oct_prm_dev, c->oct_prm.data(), sizeof(OctParams) * c->oct_prm.size(), hipMemcpyHostToDevice));
    c->view.bvh = d_nodes;
    c->view.tri = d_tri;
    c->view.prim_n = d_pn;
    c->view.prim_light = d_pl;
    c->view.mats = d_mats;
    c->view.lights = d_lights;
    c->view.light_cdf = d_cdf;
    c->view.light_guide = d_guide;
    c->forest_depth = depth;
    // the shallowest stack that holds every tree's deepest descent
    if (c->cfg.stack <= depth) c->cfg.stack = depth < 32 ? 32 : (depth < 48 ? 48 : 64);
    neb_status st = restart(c, nullptr);
    if (st != NEB_OK) return st;
    HIP_TRY(hipDeviceSynchronize());
    c->ready = true;
    return NEB_OK;
}

extern "C" neb_status neb_set_batch_scene(neb_ctx c, int32_t scene, const float* vertices, int32_t nv,
                                          const int32_t* tris, const int32_t* tri_material, int32_t nt,
                                          const neb_material* materials, int32_t nm,
                                          const neb_point_light* point_lights, int32_t npl, const neb_camera* camera) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (scene < 0 || scene >= c->n_scenes) return fail(NEB_ERR_INVALID_ARG, "scene index out of range");
    HostScene H;
    neb_status st = build_host_scene(c->prm[scene], vertices, nv, tris, tri_material, nt, materials, nm, point_lights,
                                     npl, camera, H);
    if (st != NEB_OK) return st;
    HIP_TRY(hipDeviceSynchronize());
    c->hs[scene] = std::move(H);
    c->ready = false;
    drop_graph(c);
    // a batch of one uploads at once, so that scene errors surface here
    bool all = true;
    for (const HostScene& h : c->hs) all = all && h.set;
    if (all && c->n_scenes == 1) return prepare(c);
    return NEB_OK;
}

extern "C" neb_status neb_set_scene(neb_ctx c, const float* vertices, int32_t nv, const int32_t* tris,
                                    const int32_t* tri_material, int32_t nt, const neb_material* materials, int32_t nm,
                                    const neb_point_light* point_lights, int32_t npl, const neb_camera* camera) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (c->n_scenes != 1) return fail(NEB_ERR_STATE, "neb_set_scene needs a context of one scene");
    return neb_set_batch_scene(c, 0, vertices, nv, tris, tri_material, nt, materials, nm, point_lights, npl, camera);
}

static RenderArgs make_args(neb_ctx c) {
    RenderArgs A;
    A.S = c->view;
    A.sc = c->sc_dev;
    A.pix_base = c->pix_base_dev;
    A.cnt = c->cnt;
    A.n_scenes = c->n_scenes;
    A.L = c->L;
    A.npix = c->npix;
    A.photons = c->photons;
    A.density_mode = c->density_mode;
    A.lp_base = c->lp_base_dev;
    A.n_lp = c->n_lp;
    A.dg = c->dg;
    A.ng = c->ng;
    A.recycle = c->recycle;
    return A;
}

template <int kStack>
static void launch_extend(neb_ctx c, int64_t cap, const float4* org, const float4* dir, int32_t* count, int32_t* next,
                          int rays, const HitBins& B, int2* hits, hipStream_t s) {
    hipLaunchKernelGGL((k_extend<kStack, false>), dim3(trace_grid(c, cap, c->cfg.trace_bpc)), dim3(kTraceBlock), 0, s,
                       c->view, (const SceneInfo*)c->sc_dev, org, dir, (const int32_t*)count, next, hits, rays,
                       c->cnt, B, (const float*)nullptr, (int32_t*)nullptr,
                       rays == 0 ? c->cnt->cam_next : c->cnt->trace_next,
                       rays == 0 ? &c->cnt->cam_done : &c->cnt->trace_done);
}

// the queued NEE shadow rays, any-hit, with the NEE launch shape
template <int kStack>
static void launch_shadow(neb_ctx c, hipStream_t s) {
    hipLaunchKernelGGL((k_extend<kStack, true>), dim3(trace_grid(c, c->vcap, c->cfg.nee_bpc)), dim3(kTraceBlock), 0, s,
                       c->view, (const SceneInfo*)c->sc_dev, (const float4*)c->sq0, (const float4*)c->sq1,
                       (const int32_t*)&c->cnt->n_shadow, (int32_t*)nullptr, (int2*)nullptr, 2, c->cnt, HitBins{},
                       (const float*)c->sqt, c->svis, c->cnt->trace_next, &c->cnt->trace_done);
}

// rays: 0 counts camera rays (the camera pass, which has work counters of
// its own: it may run beside the photon bounces), 1 photon rays
static void extend(neb_ctx c, int64_t cap, const float4* org, const float4* dir, int32_t* count, int32_t* next,
                   int rays, hipStream_t s, bool bin, int2* hits) {
    HitBins B{};
    if (bin) {
        B.bin = c->pbin;
        B.count = c->bcount;
        B.prm = c->oct_prm_dev;
        B.bits = c->bin_bits;
        B.n_bins = c->n_bins;
    }
    if (c->cfg.stack == 32) launch_extend<32>(c, cap, org, dir, count, next, rays, B, hits, s);
    else if (c->cfg.stack == 48) launch_extend<48>(c, cap, org, dir, count, next, rays, B, hits, s);
    else launch_extend<64>(c, cap, org, dir, count, next, rays, B, hits, s);
}

// NEE, first part: light samples and the shadow-ray queue, then the shadow
// rays (they need the vertices only, not rho)
static void nee_rays(neb_ctx c, const RenderArgs& A, hipStream_t s) {
    const int grid = grid_of(c->vcap, kNeeBlock);
    hipLaunchKernelGGL(k_nee_rays, dim3(grid), dim3(kNeeBlock), 0, s, A, c->V, (const int32_t*)c->nvtx,
                       c->sq0, c->sq1, c->sqt, &c->cnt->n_shadow);
    if (c->cfg.stack == 32) launch_shadow<32>(c, s);
    else if (c->cfg.stack == 48) launch_shadow<48>(c, s);
    else launch_shadow<64>(c, s);
}

// NEE, second part: contributions and NEB photons (needs rho)
static void nee_finish(neb_ctx c, const RenderArgs& A, Images im, hipStream_t s) {
    hipLaunchKernelGGL(k_nee_finish, dim3(grid_of(c->vcap, kNeeBlock)), dim3(kNeeBlock), 0, s, A, c->V,
                       (const int32_t*)c->nvtx, (const int32_t*)c->svis, im, c->pq[0],
                       &c->cnt->pcount[0]);
}

// Pass 1 of an iteration: camera paths traced and shaded into the vertex
// and event stores of the given parity.  It reads nothing of the iteration
// before, so it may run on its own stream beside that iteration's photon
// bounces (its queues, hits and work counters are its own).
static void enqueue_camera(neb_ctx c, hipStream_t s, int parity, bool record) {
    RenderArgs A = make_args(c);
    const int npix = c->npix, L = c->L;
    Counters* cnt = c->cnt;
    hipLaunchKernelGGL(k_cam_begin, dim3(1), dim3(1), 0, s, cnt, parity);
    if (c->slots)
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(c->slot_cap, 256)), dim3(256), 0, s, c->slots, -1, c->slot_cap);
    if (record)
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of((int64_t)npix * L * 6, 256)), dim3(256), 0, s, (int32_t*)c->recs, 0,
                           (int64_t)npix * L * 6);
    TIMED(K_CAMERA, hipLaunchKernelGGL(k_camera, dim3(grid_of(npix, kCameraBlock)), dim3(kCameraBlock), 0, s, A,
                                       c->q[0]));
    for (int k = 1; k <= L; ++k) {
        int in = (k - 1) & 1, out = k & 1;
        TIMED(K_EXTEND_CAMERA, extend(c, npix, c->q[in].q0, c->q[in].q1, &cnt->qcount[in], &cnt->qcount[out], 0, s,
                                      false, c->chits));
        TIMED(K_SHADE, hipLaunchKernelGGL(k_shade, dim3(grid_of(npix, kShadeBlock)), dim3(kShadeBlock), 0, s, A, c->q[in],
                                          &cnt->qcount[in], c->chits, c->q[out], &cnt->qcount[out], c->Vb[parity],
                                          &cnt->n_vertices[parity], c->ev0b[parity], c->ev1b[parity],
                                          &cnt->n_events[parity], c->slots,
                                          record ? c->recs : (neb_path_record*)nullptr));
    }
}

// the camera pass of the given parity on the third stream, after the work
// queued on s so far
static hipError_t fork_camera(neb_ctx c, hipStream_t s, int parity) {
    hipError_t e = hipEventRecord(c->ev_cam_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->cam, c->ev_cam_fork, 0);
    if (e != hipSuccess) return e;
    enqueue_camera(c, c->cam, parity, false);
    return hipEventRecord(c->ev_cam_done, c->cam);
}

// Enqueues one iteration.  Every argument is fixed for the context (the
// iteration number is read from device memory), so the same sequence can be
// captured once and replayed.  parity picks the vertex and event stores;
// cam_inline: the camera pass is enqueued here (else it ran beside the
// iteration before); next: the next iteration's camera pass is forked onto
// the third stream and joined at the end.
static neb_status enqueue_iteration(neb_ctx c, hipStream_t s, int parity, bool cam_inline, bool next, bool record) {
    RenderArgs A = make_args(c);
    const int npix = c->npix, L = c->L;
    const int64_t vcap = c->vcap;
    Counters* cnt = c->cnt;
    Images im{c->img, c->img + 3 * (size_t)npix, c->img + 6 * (size_t)npix, c->img + 9 * (size_t)npix};
    c->V = c->Vb[parity];
    c->ev0 = c->ev0b[parity];
    c->ev1 = c->ev1b[parity];
    c->nvtx = &cnt->n_vertices[parity];
    c->nevt = &cnt->n_events[parity];
    int32_t* const nv = c->nvtx;
    if (!c->side) {
        HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        HIP_TRY(hipStreamCreateWithFlags(&c->cam, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&c->ev_nee, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&c->ev_cam_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&c->ev_cam_done, hipEventDisableTiming));
        for (auto& e : c->ev_merge) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    // learned density: train on the octree in iterations 1..T, then use the model
    const int it = c->iter + 1;
    const int T = c->mlp_mode ? c->mcfg.train_iterations : 0;
    const bool model = c->mlp_mode && it > T;
    if (cam_inline) enqueue_camera(c, s, parity, record);
    hipLaunchKernelGGL(k_iter_begin, dim3(1), dim3(1), 0, s, cnt, c->oct_dyn, c->mlp_mode ? T : INT32_MAX);
    // The next iteration's camera pass writes the other parity's stores
    // (pass 3 of the iteration before read them, and it is done) and its own
    // queues, so it may start now, beside all of this iteration but its
    // camera pass; with single-thread deposits it also refills the deposit
    // slots, so it waits for this iteration's deposits.
    if (next && !c->slots) HIP_TRY(fork_camera(c, s, parity ^ 1));
    // bounces: NEB photons make at most maxlen - 2 segments, light photons maxlen - 1
    const bool lp = c->n_lp > 0;
    const int rounds = std::max((c->photons && L >= 3) ? L - 2 : 0, lp ? L - 1 : 0);
    // NEE's shadow rays and the merge grid need only this iteration's
    // vertices: they run on the side stream while the octree deposits and
    // the density (latency bound, the chip half idle) run here.
    // the second stream, or the caller's when the launches are serialised
    hipStream_t t = c->cfg.concurrent ? c->side : s;
    HIP_TRY(hipEventRecord(c->ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(t, c->ev_fork, 0));
    prof_begin(c, K_NEE, t);
    nee_rays(c, A, t);
    prof_end(c, t);
    HIP_TRY(hipEventRecord(c->ev_nee, t));
    if (rounds > 0) {
        hipStream_t g = t;
        int64_t n = (int64_t)c->G.T * c->G.D + 1;
        prof_begin(c, K_GRID_BUILD, g);
        hipLaunchKernelGGL(k_grid_count, dim3(grid_of(vcap, 256)), dim3(256), 0, g, (const neb_material*)c->view.mats,
                           (const SceneInfo*)c->sc_dev, c->V, (const int32_t*)nv, c->G);
        scan_exclusive(c->G.count, c->G.start, n, c->G.sums, g, true);
        hipLaunchKernelGGL(k_grid_scatter, dim3(grid_of(vcap, 256)), dim3(256), 0, g,
                           (const neb_material*)c->view.mats, (const SceneInfo*)c->sc_dev, c->V,
                           (const int32_t*)nv, c->G);
        prof_end(c, g);
    }
    // deposits of this iteration's NEE vertices into their scenes' octrees
    const bool set_mode = c->density_mode == NEB_DENSITY_RADIUS || c->density_mode == NEB_DENSITY_KNN;
    // without NEB photons rho enters nothing (flux, MIS), so the density
    // stage is skipped (the learned density still trains on it)
    const bool need_rho = c->photons || c->mlp_mode;
    if (!need_rho) {
    } else if (set_mode) {
        // density grid over this iteration's NEE vertices
        prof_begin(c, K_DENSITY_GRID, s);
        hipLaunchKernelGGL(k_dgrid_count, dim3(grid_of(vcap, 256)), dim3(256), 0, s, (const SceneInfo*)c->sc_dev, c->V,
                           (const int32_t*)nv, c->dg, 0);
        scan_exclusive(c->dg.count, c->dg.start, (int64_t)c->dg.T + 1, c->dg.sums, s);
        hipLaunchKernelGGL(k_dgrid_scatter, dim3(grid_of(vcap, 256)), dim3(256), 0, s, (const SceneInfo*)c->sc_dev,
                           c->V, (const int32_t*)nv, c->dg, 0);
        prof_end(c, s);
    } else if (c->density_mode != NEB_DENSITY_ANALYTIC && !model) {
        hipError_t e;
        const float* pos = (const float*)c->V.v0;
        const int32_t* tagw = (const int32_t*)c->V.v1 + 3;
        prof_begin(c, K_OCTREE_INSERT, s);
        if (c->slots)
            e = octree_insert_single(c->oct_nodes, c->oct_states, c->oct_prm_dev, c->oct_dyn, pos, 4, tagw, 8, c->slots,
                                     (int32_t)c->slot_cap, s);
        else
            e = octree_insert_rounds(c->oct_nodes, c->oct_states, c->oct_prm_dev, c->oct_dyn, pos, 4, tagw, 8,
                                     nv, (int32_t)vcap, c->defer, c->defer_cnt, s);
        prof_end(c, s);
        HIP_TRY(e);
    }
    if (next && c->slots) HIP_TRY(fork_camera(c, s, parity ^ 1));
    // pass 2
    if (model) {
        const OctParams& P0 = c->oct_prm[0];
        prof_begin(c, K_DENSITY, s);
        HIP_TRY(mlp_infer(c->mlp, (const float*)c->V.v0, 4, (const float*)c->V.v1, 4, nv,
                          (int32_t)vcap, &P0, c->V.rho, 1, s));
        const int j = it - T;
        if (j == 1 || (j - 1) % c->mcfg.probe_every == 0) {
            hipLaunchKernelGGL(k_mlp_probe, dim3(grid_of(vcap, 256, 4096)), dim3(256), 0, s, c->V,
                               (const int32_t*)nv, (const int32_t*)c->oct_nodes,
                               (const OctState*)c->oct_states, P0, (const OctDyn*)c->oct_dyn, j == 1 ? 1 : 0,
                               c->mcfg.probes, c->mcfg.seed, 0x50524F42u, (const Counters*)cnt, c->reg_total,
                               c->reg_bad, c->reg_sum, c->mcfg.max_rel_error, c->mlp_cnt);
            hipLaunchKernelGGL(k_mlp_clear_gate_counts, dim3(1), dim3(1), 0, s, c->mlp_cnt);
            hipLaunchKernelGGL(k_mlp_gate, dim3(grid_of(kRegions, 256)), dim3(256), 0, s, (const int32_t*)c->reg_total,
                               (const int32_t*)c->reg_bad, (const float*)c->reg_sum, c->mcfg.max_rel_error,
                               c->reg_gate, c->mlp_cnt);
        }
        hipLaunchKernelGGL(k_density_fallback, dim3(grid_of(vcap, 256)), dim3(256), 0, s, c->V,
                           (const int32_t*)nv, (const int32_t*)c->reg_gate,
                           (const int32_t*)c->oct_nodes, (const OctState*)c->oct_states, P0,
                           (const OctDyn*)c->oct_dyn, c->mlp_cnt);
        prof_end(c, s);
    } else if (need_rho) {
        TIMED(K_DENSITY, hipLaunchKernelGGL(k_density, dim3(grid_of(vcap, 256)), dim3(256), 0, s, A, c->V,
                                            (const int32_t*)nv, (const int32_t*)c->oct_nodes,
                                            (const OctState*)c->oct_states, (const OctParams*)c->oct_prm_dev,
                                            (const OctDyn*)c->oct_dyn));
    }
    // NEE recycling: the vertices by cells of the recycling radius and n_E
    if (c->recycle) {
        prof_begin(c, K_NEE_RECYCLE, s);
        hipLaunchKernelGGL(k_dgrid_count, dim3(grid_of(vcap, 256)), dim3(256), 0, s, (const SceneInfo*)c->sc_dev, c->V,
                           (const int32_t*)nv, c->ng, 1);
        scan_exclusive(c->ng.count, c->ng.start, (int64_t)c->ng.T + 1, c->ng.sums, s);
        hipLaunchKernelGGL(k_dgrid_scatter, dim3(grid_of(vcap, 256)), dim3(256), 0, s, (const SceneInfo*)c->sc_dev,
                           c->V, (const int32_t*)nv, c->ng, 1);
        hipLaunchKernelGGL(k_nee_count, dim3(grid_of(vcap, 256)), dim3(256), 0, s, A, c->V,
                           (const int32_t*)nv);
        prof_end(c, s);
    }
    // light photons take the first entries of photon queue 0, the NEB photons follow
    if (lp)
        TIMED(K_LIGHT_PHOTON, hipLaunchKernelGGL(k_lp_emit, dim3(grid_of(c->n_lp, 256)), dim3(256), 0, s, A,
                                                 c->pq[0], &cnt->pcount[0]));
    HIP_TRY(hipStreamWaitEvent(s, c->ev_nee, 0));
    TIMED(K_NEE, nee_finish(c, A, im, s));
    if (c->recycle)
        TIMED(K_NEE_RECYCLE, hipLaunchKernelGGL(k_nee_recycle, dim3(grid_of(vcap, 256)), dim3(256), 0, s, A, c->V,
                                                (const int32_t*)nv, im));
    const int64_t pcap = c->pcap;
    if (rounds > 0) {
        // the merge grid comes from the second stream, whose order puts it
        // before every merge launch: the first bounce's closest hits and
        // scatter need not wait for it.  (The shadow rays, the only other
        // closest-hit launch there, are done: NEE's contributions waited
        // for them; closest-hit launches share their work counters.)
        const int pgrid = c->cfg.photon_bpc > 0 ? std::max(1, std::min(grid_of(pcap, 64, 1 << 20), c->cus * c->cfg.photon_bpc))
                                                : grid_of(pcap, 256);
        for (int j = 1; j <= rounds; ++j) {
            // bounce j reads queue `in` (and writes its hits), its scatter fills `out`
            const int in = (j - 1) % kPhotonBufs, out = j % kPhotonBufs;
            int2* hj = c->phits[in];
            const bool ordered = c->cfg.photon_order != 0;
            TIMED(K_EXTEND_PHOTON, extend(c, pcap, c->pq[in].p0, c->pq[in].p1, &cnt->pcount[in], &cnt->pcount[out],
                                          1, s, ordered, hj));
            if (j == 1 && lp)
                TIMED(K_LIGHT_PHOTON,
                      hipLaunchKernelGGL(k_lp_first, dim3(grid_of(c->n_lp, 256)), dim3(256), 0, s, A, c->pq[0], hj,
                                         (const int32_t*)c->oct_nodes, (const OctState*)c->oct_states,
                                         (const OctParams*)c->oct_prm_dev, (const OctDyn*)c->oct_dyn));
            if (ordered) {
                // photons in the spatial order of their hits; the order array
                // is shared, so the merges of the bounce before must be done
                if (j > 1) HIP_TRY(hipStreamWaitEvent(s, c->ev_merge[j - 1], 0));
                prof_begin(c, K_PHOTON_ORDER, s);
                scan_exclusive(c->bcount, c->bstart, c->n_bins + 1, c->bsums, s);
                hipLaunchKernelGGL(k_bin_scatter, dim3(grid_of(pcap, 256)), dim3(256), 0, s, (const int32_t*)c->pbin,
                                   (const int32_t*)&cnt->pcount[in], c->bcount, (const int32_t*)c->bstart, c->porder);
                prof_end(c, s);
            }
            // queue `out` was the input of bounce j + 1 - kPhotonBufs: its merges
            // must be done before the scatter overwrites it
            if (j + 1 - kPhotonBufs >= 1) HIP_TRY(hipStreamWaitEvent(s, c->ev_merge[j + 1 - kPhotonBufs], 0));
            TIMED(K_PHOTON_SCATTER,
                  hipLaunchKernelGGL(k_pscatter, dim3(grid_of(pcap, kScatterBlock)), dim3(kScatterBlock), 0, s, A,
                                     c->pq[in], (const int32_t*)&cnt->pcount[in], (const int2*)hj, c->pq[out],
                                     &cnt->pcount[out], &cnt->mcount[in]));
            // the merges of bounce j on the second stream, beside the closest
            // hits and scatters of the bounces after it
            HIP_TRY(hipEventRecord(c->ev_fork, s));
            HIP_TRY(hipStreamWaitEvent(t, c->ev_fork, 0));
            prof_begin(c, K_PHOTON, t);
            hipLaunchKernelGGL(k_photon, dim3(pgrid), dim3(64), 0, t, A, c->pq[in], (const int32_t*)&cnt->mcount[in],
                               (const int2*)hj, c->G, im,
                               ordered ? (const int32_t*)c->porder : (const int32_t*)nullptr);
            prof_end(c, t);
            HIP_TRY(hipEventRecord(c->ev_merge[j], t));
        }
        HIP_TRY(hipStreamWaitEvent(s, c->ev_merge[rounds], 0));
    }
    // pass 3
    TIMED(K_FINALIZE, hipLaunchKernelGGL(k_finalize, dim3(grid_of(c->ecap, 256)), dim3(256), 0, s, A,
                                         (const float4*)c->ev0, (const float4*)c->ev1,
                                         (const int32_t*)c->nevt, (const float*)c->V.rho,
                                         (const float*)c->V.ne, im));
    hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(1), 0, s, cnt, parity);
    if (next) HIP_TRY(hipStreamWaitEvent(s, c->ev_cam_done, 0));
    // learned density, training iterations: this iteration's vertices with
    // rho > 0 form the pool, then Adam steps on batches drawn from it
    if (c->mlp_mode && !model) {
        const OctParams& P0 = c->oct_prm[0];
        const neb_mlp_params& M = c->mcfg;
        prof_begin(c, K_MLP_TRAIN, s);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, c->tcount, 0, (int64_t)1);
        hipLaunchKernelGGL(k_mlp_collect, dim3(grid_of(vcap, 256)), dim3(256), 0, s, c->V,
                           (const int32_t*)nv, c->tpos, c->tnrm, c->ttgt, c->tcount);
        if (it == 1 && !c->mlp_given) HIP_TRY(mlp_norm_from_pool(c->mlp, c->ttgt, c->tcount, (int32_t)vcap, s));
        hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, s, c->mlp.loss, 0.f, (int64_t)1);
        for (int k = 0; k < M.steps_per_iteration; ++k) {
            HIP_TRY(mlp_gradient(c->mlp, c->tpos, 3, c->tnrm, 3, c->ttgt, c->tcount, (int32_t)vcap, M.batch, 1, M.seed,
                                 0x4D4C5031u, &P0, s));
            HIP_TRY(mlp_adam(c->mlp, M.lr, M.beta1, M.beta2, M.eps, s));
        }
        prof_end(c, s);
        c->last_train_steps = M.steps_per_iteration;
    }
    HIP_TRY(hipGetLastError());
    return NEB_OK;
}

// captures one iteration (of the given parity and camera-pass placement) on
// a private stream into an executable graph
static neb_status capture(neb_ctx c, int parity, bool cam_inline, bool next, int key) {
    if (c->gexec[key]) return NEB_OK;
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    bool was = c->prof_on;
    c->prof_on = false;
    neb_status st = enqueue_iteration(c, c->cap_stream, parity, cam_inline, next, false);
    c->prof_on = was;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != NEB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(NEB_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(NEB_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    c->graph[key] = g;
    c->gexec[key] = x;
    return NEB_OK;
}

// Iteration k of the call uses the stores of parity k & 1.  With the second
// stream on, each iteration but the last forks the next one's camera pass;
// the last joins everything, so nothing is in flight between calls.  (The
// learned density's training, probes and fallback read only the current
// parity's stores and the model's own buffers, so its iterations overlap
// the same way; they are launched eagerly, since they differ from one
// another.)
// The eager sequence of a whole call: iteration k uses parity k & 1 and,
// but for the last, forks the next iteration's camera pass.
static neb_status enqueue_call(neb_ctx c, int32_t n_iterations, hipStream_t s) {
    bool cam_done = false;
    for (int i = 0; i < n_iterations; ++i) {
        const bool next = i + 1 < n_iterations && c->cfg.concurrent;
        neb_status st = enqueue_iteration(c, s, i & 1, !cam_done, next, false);
        if (st != NEB_OK) return st;
        cam_done = next;
    }
    return NEB_OK;
}

// the graph of a whole call of n_iterations (captured on first use; the
// last kCallGraphs counts are kept)
static neb_status call_graph(neb_ctx c, int32_t n_iterations, hipGraphExec_t* out) {
    for (int k = 0; k < neb_ctx_s::kCallGraphs; ++k)
        if (c->call_exec[k] && c->call_n[k] == n_iterations) {
            *out = c->call_exec[k];
            return NEB_OK;
        }
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    neb_status st = enqueue_call(c, n_iterations, c->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != NEB_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (st != NEB_OK) return st;
        return fail(NEB_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(NEB_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    const int k = c->call_next;
    c->call_next = (k + 1) % neb_ctx_s::kCallGraphs;
    if (c->call_exec[k]) (void)hipGraphExecDestroy(c->call_exec[k]);
    if (c->call_graph[k]) (void)hipGraphDestroy(c->call_graph[k]);
    c->call_graph[k] = g;
    c->call_exec[k] = x;
    c->call_n[k] = n_iterations;
    *out = x;
    return NEB_OK;
}

static neb_status render_n(neb_ctx c, int32_t n_iterations, hipStream_t s) {
    const bool record_pending = c->recs && c->first_iter_recorded == 0;
    if (c->use_graph == 2 && n_iterations > 0 && !c->prof_on && !record_pending && !c->mlp_mode) {
        hipGraphExec_t x = nullptr;
        neb_status st = call_graph(c, n_iterations, &x);
        if (st != NEB_OK) return st;
        HIP_TRY(hipGraphLaunch(x, s));
        c->iter += n_iterations;
        return NEB_OK;
    }
    bool cam_done = false;  // this iteration's camera pass ran beside the iteration before
    for (int i = 0; i < n_iterations; ++i) {
        const int parity = i & 1;
        const bool record = c->recs && c->first_iter_recorded == 0 && !cam_done;
        const bool next = i + 1 < n_iterations && c->cfg.concurrent;
        if (c->use_graph == 1 && !c->prof_on && !record && !c->mlp_mode) {
            const int key = 4 * parity + 2 * (cam_done ? 0 : 1) + (next ? 1 : 0);
            neb_status st = capture(c, parity, !cam_done, next, key);
            if (st != NEB_OK) return st;
            HIP_TRY(hipGraphLaunch(c->gexec[key], s));
        } else {
            neb_status st = enqueue_iteration(c, s, parity, !cam_done, next, record);
            if (st != NEB_OK) return st;
        }
        c->iter += 1;
        if (record) c->first_iter_recorded = c->iter;
        cam_done = next;
    }
    return NEB_OK;
}

extern "C" neb_status neb_render(neb_ctx c, int32_t n_iterations, void* stream) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (n_iterations < 0) return fail(NEB_ERR_INVALID_ARG, "negative iteration count");
    neb_status st = prepare(c);
    if (st != NEB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    return render_n(c, n_iterations, s);
}

// iterations scene s has taken part in
static int scene_iters(neb_ctx c, int s) {
    int spp = c->prm[s].spp;
    return spp > 0 ? std::min(c->iter, spp) : c->iter;
}

static neb_status copy_out(const float* src_dev, float* dst, int32_t is_dev, float scale, hipStream_t s, int64_t n) {
    if (is_dev) {
        hipLaunchKernelGGL(k_scale_image, dim3(grid_of(n, 256)), dim3(256), 0, s, src_dev, dst, n, scale);
        HIP_TRY(hipGetLastError());
        return NEB_OK;
    }
    std::vector<float> h((size_t)n);
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(h.data(), src_dev, n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) dst[i] = h[i] * scale;
    return NEB_OK;
}

static neb_status check_scene_ready(neb_ctx c, int32_t scene) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (scene < 0 || scene >= c->n_scenes) return fail(NEB_ERR_INVALID_ARG, "scene index out of range");
    if (!c->ready) return fail(NEB_ERR_STATE, "scenes not set or not rendered since they changed");
    return NEB_OK;
}

extern "C" neb_status neb_get_scene_image(neb_ctx c, int32_t scene, float* rgb, int32_t is_dev, void* stream) {
    if (!rgb) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    neb_status st = check_scene_ready(c, scene);
    if (st != NEB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = 3 * (int64_t)c->prm[scene].width * c->prm[scene].height;
    const int64_t N = 3 * (int64_t)c->npix, off = 3 * (int64_t)c->pix_base[scene];
    int it = scene_iters(c, scene);
    float scale = it > 0 ? 1.0f / (float)it : 0.f;
    if (is_dev) {
        hipLaunchKernelGGL(k_mean_image, dim3(grid_of(n, 256)), dim3(256), 0, s, c->img + off, c->img + N + off,
                           c->img + 2 * N + off, c->img + 3 * N + off, rgb, n, scale);
        HIP_TRY(hipGetLastError());
        return NEB_OK;
    }
    std::vector<float> h(4 * (size_t)n);
    HIP_TRY(hipStreamSynchronize(s));
    for (int t = 0; t < 4; ++t)
        HIP_TRY(hipMemcpy(h.data() + t * n, c->img + t * N + off, n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) rgb[i] = (h[i] + h[n + i] + h[2 * n + i] + h[3 * n + i]) * scale;
    return NEB_OK;
}

extern "C" neb_status neb_get_image(neb_ctx c, float* rgb, int32_t is_dev, void* stream) {
    return neb_get_scene_image(c, 0, rgb, is_dev, stream);
}

extern "C" neb_status neb_get_scene_technique_images(neb_ctx c, int32_t scene, float* e, float* E, float* P,
                                                     int32_t is_dev, void* stream) {
    neb_status st = check_scene_ready(c, scene);
    if (st != NEB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = 3 * (int64_t)c->prm[scene].width * c->prm[scene].height;
    const int64_t N = 3 * (int64_t)c->npix, off = 3 * (int64_t)c->pix_base[scene];
    int it = scene_iters(c, scene);
    float scale = it > 0 ? 1.0f / (float)it : 0.f;
    float* dst[3] = {e, E, P};
    for (int t = 0; t < 3; ++t)
        if (dst[t]) {
            st = copy_out(c->img + t * N + off, dst[t], is_dev, scale, s, n);
            if (st != NEB_OK) return st;
        }
    return NEB_OK;
}

extern "C" neb_status neb_get_technique_images(neb_ctx c, float* e, float* E, float* P, int32_t is_dev, void* stream) {
    return neb_get_scene_technique_images(c, 0, e, E, P, is_dev, stream);
}

static neb_status check_point_density(const float* points, int32_t n, const float* queries, int32_t n_query,
                                      int32_t mode, float radius, int32_t k, float* out) {
    if (n < 0 || n_query < 0) return fail(NEB_ERR_INVALID_ARG, "negative size");
    if (mode != NEB_DENSITY_RADIUS && mode != NEB_DENSITY_KNN) return fail(NEB_ERR_INVALID_ARG, "mode must be 4 or 5");
    if (!(radius > 0.f) || !std::isfinite(radius)) return fail(NEB_ERR_INVALID_ARG, "radius must be > 0");
    if (mode == NEB_DENSITY_KNN && (k < 1 || k > kKnnMax)) return fail(NEB_ERR_INVALID_ARG, "k out of range (1 .. 16)");
    if (n_query > 0 && (!queries || !out || (n > 0 && !points))) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    return NEB_OK;
}

// buckets of the point-set grid for n points
static int32_t pset_buckets(int32_t n) {
    return (int32_t)std::max<uint64_t>(1024, std::min<uint64_t>(next_pow2((uint64_t)std::max(n, 1)) / 2, 1u << 23));
}

// grid over the points (count, scan, scatter) and the queries, in stream order
static void pset_enqueue(const DGrid& D, const float* points, int32_t n, const float* queries, int32_t n_query,
                         int32_t mode, float radius, int32_t k, float* out, hipStream_t s) {
    const float inv_cell = 1.0f / (2.0001f * radius);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_of((int64_t)D.T + 1, 256)), dim3(256), 0, s, D.count, 0,
                       (int64_t)D.T + 1);
    if (n > 0) hipLaunchKernelGGL(k_pset_count, dim3(grid_of(n, 256)), dim3(256), 0, s, points, n, inv_cell, D);
    scan_exclusive(D.count, D.start, (int64_t)D.T + 1, D.sums, s);
    if (n > 0) hipLaunchKernelGGL(k_pset_scatter, dim3(grid_of(n, 256)), dim3(256), 0, s, points, n, inv_cell, D);
    hipLaunchKernelGGL(k_pset_query, dim3(grid_of(n_query, 256)), dim3(256), 0, s, queries, n_query, D, radius, inv_cell,
                       (int)mode, (int)k, out);
}

extern "C" neb_status neb_point_density(const float* points, int32_t n, const float* queries, int32_t n_query,
                                        int32_t mode, float radius, int32_t k, float* out, void* stream) {
    neb_status st = check_point_density(points, n, queries, n_query, mode, radius, k, out);
    if (st != NEB_OK || n_query == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    DGrid D{};
    D.T = pset_buckets(n);
    std::vector<void*> tmp;
    hipError_t e = dalloc(tmp, &D.count, (size_t)D.T + 1);
    if (e == hipSuccess) e = dalloc(tmp, &D.start, (size_t)D.T + 1);
    if (e == hipSuccess) e = dalloc(tmp, &D.pts, (size_t)std::max(n, 1));
    if (e == hipSuccess) e = dalloc(tmp, &D.sums, (size_t)scan_scratch((int64_t)D.T + 1));
    if (e != hipSuccess) {
        free_list(tmp);
        return oom_or_device(e, "neb_point_density");
    }
    pset_enqueue(D, points, n, queries, n_query, mode, radius, k, out, s);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    free_list(tmp);
    if (e != hipSuccess) return oom_or_device(e, "neb_point_density");
    return NEB_OK;
}

// ---------------------------------------------------------------------------
// The point-set densities without allocation: the grid of
// neb_point_density lives in `scratch`, a fixed device array of its own on
// every device, for callers that cannot allocate.  Its layout: bucket counts
// and starts (kScratchBuckets + 1 ints each), the scan's block sums, then
// the points in bucket order (float4, 256-byte aligned).
// ---------------------------------------------------------------------------
constexpr int32_t kScratchMaxPoints = 1 << 19;
constexpr int32_t kScratchBuckets = 1 << 18;  // pset_buckets(kScratchMaxPoints)
constexpr int64_t scan_scratch_c(int64_t n) {
    int64_t tot = 0;
    while (n > 1) {
        n = (n + kScanTile - 1) / kScanTile;
        tot += n;
    }
    return tot > 1 ? tot : 1;
}
constexpr size_t kScratchIntBytes =
    ((4 * (2 * ((size_t)kScratchBuckets + 1) + (size_t)scan_scratch_c((int64_t)kScratchBuckets + 1))) + 255) & ~(size_t)255;
constexpr size_t kScratchBytes = kScratchIntBytes + 16 * (size_t)kScratchMaxPoints;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's `scratch` (the name is a host-side stand-in
// in host code), looked up once per device with that device current.
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[256];

static neb_status scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return oom_or_device(e, "hipGetDevice");
    if (dev < 0 || dev >= 256) return fail(NEB_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(NEB_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                                   hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NEB_OK;
}

extern "C" neb_status neb_point_density_noalloc(const float* points, int32_t n, const float* queries,
                                                int32_t n_query, int32_t mode, float radius, int32_t k, float* out,
                                                void* stream) {
    neb_status st = check_point_density(points, n, queries, n_query, mode, radius, k, out);
    if (st != NEB_OK) return st;
    if (n > kScratchMaxPoints)
        return fail(NEB_ERR_CAPACITY, "neb_point_density_noalloc takes at most 524288 points (" +
                                          std::to_string(n) + " given)");
    if (n_query == 0) return NEB_OK;
    void* base = nullptr;
    st = scratch_address(&base);
    if (st != NEB_OK) return st;
    DGrid D{};
    D.T = pset_buckets(n);
    int32_t* ints = reinterpret_cast<int32_t*>(base);
    D.count = ints;
    D.start = ints + ((size_t)kScratchBuckets + 1);
    D.sums = ints + 2 * ((size_t)kScratchBuckets + 1);
    D.pts = reinterpret_cast<float4*>(reinterpret_cast<unsigned char*>(base) + kScratchIntBytes);
    pset_enqueue(D, points, n, queries, n_query, mode, radius, k, out, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return oom_or_device(e, "neb_point_density_noalloc");
    return NEB_OK;
}

extern "C" neb_status neb_get_scene_light_photon_image(neb_ctx c, int32_t scene, float* LP, int32_t is_dev,
                                                       void* stream) {
    if (!LP) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    neb_status st = check_scene_ready(c, scene);
    if (st != NEB_OK) return st;
    const int64_t n = 3 * (int64_t)c->prm[scene].width * c->prm[scene].height;
    const int64_t N = 3 * (int64_t)c->npix, off = 3 * (int64_t)c->pix_base[scene];
    int it = scene_iters(c, scene);
    return copy_out(c->img + 3 * N + off, LP, is_dev, it > 0 ? 1.0f / (float)it : 0.f, (hipStream_t)stream, n);
}

extern "C" neb_status neb_query_density(neb_ctx c, const float* pos, const float* nrm, int32_t n, float* out,
                                        int32_t is_dev, void* stream) {
    if (!c || !pos || !nrm || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (n < 0) return fail(NEB_ERR_INVALID_ARG, "negative count");
    neb_status st0 = check_scene_ready(c, 0);
    if (st0 != NEB_OK) return st0;
    if (n == 0) return NEB_OK;
    hipStream_t s = (hipStream_t)stream;
    const OctParams& P = c->oct_prm[0];
    if (is_dev) {
        HIP_TRY(octree_density_raw(c->oct_nodes, c->oct_states, P, c->oct_dyn, pos, nrm, n, 1, out, s));
        return NEB_OK;
    }
    float *dp = nullptr, *dn = nullptr, *dout = nullptr;
    std::vector<void*> tmp;
    hipError_t e = dalloc(tmp, &dp, 3 * (size_t)n);
    if (e == hipSuccess) e = dalloc(tmp, &dn, 3 * (size_t)n);
    if (e == hipSuccess) e = dalloc(tmp, &dout, (size_t)n);
    if (e != hipSuccess) {
        free_list(tmp);
        return oom_or_device(e, "neb_query_density");
    }
    neb_status st = NEB_OK;
    if (hipMemcpy(dp, pos, 12 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dn, nrm, 12 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess ||
        octree_density_raw(c->oct_nodes, c->oct_states, P, c->oct_dyn, dp, dn, n, 1, dout, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(out, dout, 4 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
        st = fail(NEB_ERR_DEVICE, "neb_query_density transfer failed");
    free_list(tmp);
    return st;
}

// info of the octree that owns [root, end) of a pool
static neb_status octree_info(const int32_t* pool, const OctState* state, int32_t root, int32_t end, hipStream_t s,
                              int64_t info[8]) {
    OctState st;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(&st, state, sizeof(st), hipMemcpyDeviceToHost));
    int32_t used = std::min(st.alloc, end) - root;
    std::vector<int32_t> nodes((size_t)std::max(used, 0));
    if (used > 0) HIP_TRY(hipMemcpy(nodes.data(), pool + root, 4 * (size_t)used, hipMemcpyDeviceToHost));
    int64_t leaf = 0;
    for (int32_t v : nodes)
        if (v >= 0) leaf += v & kOctCountMask;
    info[0] = end - root;
    info[1] = used;
    info[2] = st.depth;
    info[3] = leaf - (int64_t)kOctSplitFactor * (int64_t)st.block_iter_sum;
    info[4] = (int64_t)oct_deposits(st);
    info[5] = st.overflow;
    info[6] = st.rejected;
    info[7] = (int64_t)st.lost;
    return NEB_OK;
}

extern "C" neb_status neb_get_stats(neb_ctx c, neb_stats* out) {
    if (!c || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    Counters hc;
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    HIP_TRY(hipMemcpy(&hc, c->cnt, sizeof(hc), hipMemcpyDeviceToHost));
    StatLine h{};
    for (int k = 0; k < kStatStripes; ++k) {
        const StatLine& L = hc.st[k];
        h.paths += L.paths;
        h.vertices += L.vertices;
        h.photons += L.photons;
        h.photon_segments += L.photon_segments;
        h.merges += L.merges;
        h.nee_visible += L.nee_visible;
        h.events += L.events;
        h.camera_rays += L.camera_rays;
        h.shadow_rays += L.shadow_rays;
        h.photon_rays += L.photon_rays;
        h.photon_items += L.photon_items;
        h.photon_continued += L.photon_continued;
        h.grid_cells += L.grid_cells;
        h.candidates += L.candidates;
        for (int r = 0; r < 3; ++r) {
            h.bvh_nodes[r] += L.bvh_nodes[r];
            h.bvh_tris[r] += L.bvh_tris[r];
        }
        h.light_photons += L.light_photons;
    }
    std::memset(out, 0, sizeof(*out));
    out->iterations = c->iter;
    out->paths = (int64_t)h.paths;
    out->vertices = (int64_t)h.vertices;
    out->photons = (int64_t)h.photons;
    out->photon_segments = (int64_t)h.photon_segments;
    out->merges = (int64_t)h.merges;
    out->nee_visible = (int64_t)h.nee_visible;
    out->events = (int64_t)h.events;
    out->rays = (int64_t)(h.camera_rays + h.shadow_rays + h.photon_rays);
    out->camera_rays = (int64_t)h.camera_rays;
    out->shadow_rays = (int64_t)h.shadow_rays;
    out->bvh_nodes = (int64_t)(h.bvh_nodes[0] + h.bvh_nodes[1] + h.bvh_nodes[2]);
    out->bvh_tris = (int64_t)(h.bvh_tris[0] + h.bvh_tris[1] + h.bvh_tris[2]);
    out->bvh_nodes_camera = (int64_t)h.bvh_nodes[0];
    out->bvh_nodes_photon = (int64_t)h.bvh_nodes[1];
    out->bvh_nodes_shadow = (int64_t)h.bvh_nodes[2];
    out->bvh_tris_camera = (int64_t)h.bvh_tris[0];
    out->bvh_tris_photon = (int64_t)h.bvh_tris[1];
    out->bvh_tris_shadow = (int64_t)h.bvh_tris[2];
    out->photon_items = (int64_t)h.photon_items;
    out->photon_continued = (int64_t)h.photon_continued;
    out->grid_cells = (int64_t)h.grid_cells;
    out->candidates = (int64_t)h.candidates;
    out->light_photons = (int64_t)h.light_photons;
    if (c->ready) {
        // octree fields: summed over the scenes of the batch (depth: the deepest)
        for (int s = 0; s < c->n_scenes; ++s) {
            int64_t info[8];
            neb_status st = octree_info(c->oct_nodes, c->oct_states + s, c->oct_prm[s].root, c->oct_prm[s].end,
                                        c->last_stream, info);
            if (st != NEB_OK) return st;
            out->oct_capacity += info[0];
            out->oct_allocated += info[1];
            out->oct_depth = std::max<int64_t>(out->oct_depth, info[2]);
            out->oct_ledger += info[3];
            out->oct_deposits += info[4];
            out->oct_overflow += info[5];
            out->oct_rejected += info[6];
            out->oct_lost += info[7];
        }
    }
    return NEB_OK;
}

extern "C" neb_status neb_get_path_records(neb_ctx c, neb_path_record* out, int64_t n) {
    if (!c || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (!c->recs || c->first_iter_recorded == 0) return fail(NEB_ERR_STATE, "no recorded iteration");
    int64_t total = (int64_t)c->npix * c->L;
    if (n < total) return fail(NEB_ERR_CAPACITY, "record buffer too small");
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    HIP_TRY(hipMemcpy(out, c->recs, sizeof(neb_path_record) * (size_t)total, hipMemcpyDeviceToHost));
    return NEB_OK;
}

extern "C" neb_status neb_get_scene_octree(neb_ctx c, int32_t scene, int32_t* nodes, int32_t cap, int64_t info[8]) {
    if (!info) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    neb_status st = check_scene_ready(c, scene);
    if (st != NEB_OK) return st;
    const OctParams& P = c->oct_prm[scene];
    st = octree_info(c->oct_nodes, c->oct_states + scene, P.root, P.end, c->last_stream, info);
    if (st != NEB_OK) return st;
    if (nodes && cap > 0)
        HIP_TRY(hipMemcpy(nodes, c->oct_nodes + P.root, 4 * (size_t)std::min(cap, P.end - P.root),
                          hipMemcpyDeviceToHost));
    return NEB_OK;
}

extern "C" neb_status neb_get_octree(neb_ctx c, int32_t* nodes, int32_t cap, int64_t info[8]) {
    return neb_get_scene_octree(c, 0, nodes, cap, info);
}

extern "C" neb_status neb_profile_kernels(neb_ctx c, int32_t enable) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (enable) {
        HIP_TRY(prof_alloc(c));
        prof_clear(c);
    }
    c->prof_on = enable != 0;
    return NEB_OK;
}

extern "C" neb_status neb_get_kernel_profile(neb_ctx c, neb_kernel_time* out, int32_t cap, int32_t* n_out) {
    if (!c || !n_out || (!out && cap > 0)) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    prof_harvest(c);
    int n = 0;
    for (int k = 0; k < K_COUNT && n < cap; ++k) {
        if (c->prof_launches[k] == 0) continue;
        std::memset(out[n].name, 0, sizeof(out[n].name));
        std::strncpy(out[n].name, kKernelNames[k], sizeof(out[n].name) - 1);
        out[n].launches = c->prof_launches[k];
        out[n].total_ms = c->prof_ms[k];
        ++n;
    }
    *n_out = n;
    return NEB_OK;
}

extern "C" neb_status neb_reset(neb_ctx c) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    HIP_TRY(hipDeviceSynchronize());
    if (!c->ready) {
        neb_status st = prepare(c);
        if (st != NEB_OK) return st;
    } else {
        neb_status st = restart(c, nullptr);
        if (st != NEB_OK) return st;
    }
    HIP_TRY(hipDeviceSynchronize());
    return NEB_OK;
}

extern "C" neb_status neb_use_graph(neb_ctx c, int32_t mode) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (mode < 0 || mode > 2) return fail(NEB_ERR_INVALID_ARG, "graph mode must be 0, 1 or 2");
    c->use_graph = mode;
    return NEB_OK;
}

static neb_status apply_config(neb_ctx c, const neb_launch_config& cfg) {
    if (cfg.bvh_stack != 32 && cfg.bvh_stack != 48 && cfg.bvh_stack != 64)
        return fail(NEB_ERR_INVALID_ARG, "bvh_stack must be 32, 48 or 64");
    if (c->ready && cfg.bvh_stack <= c->forest_depth)
        return fail(NEB_ERR_CAPACITY, "bvh_stack must exceed the stack entries every BVH needs");
    if (cfg.trace_blocks_per_cu < -1 || cfg.trace_blocks_per_cu > lds_blocks_per_cu(cfg.bvh_stack))
        return fail(NEB_ERR_INVALID_ARG, "trace_blocks_per_cu out of range for this stack");
    if (cfg.nee_blocks_per_cu < -1 || cfg.nee_blocks_per_cu > lds_blocks_per_cu(cfg.bvh_stack))
        return fail(NEB_ERR_INVALID_ARG, "nee_blocks_per_cu out of range for this stack");
    if (cfg.photon_blocks_per_cu < 0 || cfg.photon_blocks_per_cu > 64)
        return fail(NEB_ERR_INVALID_ARG, "photon_blocks_per_cu out of range (0..64)");
    if (cfg.photon_order != 0 && cfg.photon_order != 1) return fail(NEB_ERR_INVALID_ARG, "photon_order must be 0 or 1");
    if (cfg.concurrent != 0 && cfg.concurrent != 1) return fail(NEB_ERR_INVALID_ARG, "concurrent must be 0 or 1");
    c->cfg.stack = cfg.bvh_stack;
    c->cfg.trace_bpc = cfg.trace_blocks_per_cu;
    c->cfg.nee_bpc = cfg.nee_blocks_per_cu;
    c->cfg.photon_bpc = cfg.photon_blocks_per_cu;
    c->cfg.photon_order = cfg.photon_order;
    c->cfg.concurrent = cfg.concurrent;
    drop_graph(c);
    return NEB_OK;
}

extern "C" neb_status neb_set_launch_config(neb_ctx c, const neb_launch_config* cfg) {
    if (!c || !cfg) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    return apply_config(c, *cfg);
}

extern "C" neb_status neb_get_launch_config(neb_ctx c, neb_launch_config* cfg) {
    if (!c || !cfg) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    cfg->bvh_stack = c->cfg.stack;
    const int maxb = lds_blocks_per_cu(c->cfg.stack);
    cfg->trace_blocks_per_cu = c->cfg.trace_bpc < 0 ? maxb : std::min(c->cfg.trace_bpc, maxb);
    cfg->nee_blocks_per_cu = c->cfg.nee_bpc < 0 ? maxb : std::min(c->cfg.nee_bpc, maxb);
    cfg->photon_blocks_per_cu = c->cfg.photon_bpc;
    cfg->photon_order = c->cfg.photon_order;
    cfg->concurrent = c->cfg.concurrent;
    return NEB_OK;
}

// device time of the listed kernels over n iterations with configuration cfg
static neb_status time_config(neb_ctx c, const neb_launch_config& cfg, int n, const int* kids, int nk, hipStream_t s,
                              double& ms) {
    neb_status st = apply_config(c, cfg);
    if (st != NEB_OK) return st;
    prof_clear(c);
    st = render_n(c, n, s);
    if (st != NEB_OK) return st;
    prof_harvest(c);
    ms = 0.0;
    for (int k = 0; k < nk; ++k) ms += c->prof_ms[kids[k]];
    return NEB_OK;
}

// whole iterations with the launches as they run (no event pairs around
// each launch): the span of `n` iterations on s
static neb_status time_iterations(neb_ctx c, const neb_launch_config& cfg, int n, hipStream_t s, double& ms) {
    neb_status st = apply_config(c, cfg);
    if (st != NEB_OK) return st;
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e == hipSuccess) st = render_n(c, n, s);
    if (e == hipSuccess && st == NEB_OK) e = hipEventRecord(b, s);
    if (e == hipSuccess && st == NEB_OK) e = hipEventSynchronize(b);
    float t = 0.f;
    if (e == hipSuccess && st == NEB_OK) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (st != NEB_OK) return st;
    if (e != hipSuccess) return fail(NEB_ERR_DEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
    ms = t;
    return NEB_OK;
}

// Picks the launch shapes by timing real iterations of this context:
// first the traversal stack depth and resident closest-hit blocks per CU,
// then the NEE (shadow-ray) blocks per CU, then the photon stage (order
// and merge grid), each by the time of its own kernels; then the photon
// order and the closest-hit and merge blocks per CU once more by the time
// of whole iterations with the launches as they run, since beside each
// other the shape that is fastest alone is not the iteration's (fewer
// closest-hit blocks leave the merges more of the chip).  The context is reset
// afterwards (images, statistics, octrees, iteration counter).
extern "C" neb_status neb_autotune(neb_ctx c, int32_t trial_iterations, void* stream, neb_launch_config* chosen) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (trial_iterations < 1 || trial_iterations > 64) return fail(NEB_ERR_INVALID_ARG, "trial_iterations out of range (1..64)");
    neb_status st = prepare(c);
    if (st != NEB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    HIP_TRY(prof_alloc(c));
    bool was_on = c->prof_on;
    c->prof_on = true;
    LaunchCfg keep = c->cfg;
    neb_launch_config best{c->cfg.stack, -1, -1, c->cfg.photon_bpc, c->cfg.photon_order, c->cfg.concurrent};
    st = render_n(c, 1, s);  // warm-up: octree and caches
    double best_ms = 1e300;
    const int trace_k[2] = {K_EXTEND_CAMERA, K_EXTEND_PHOTON};
    for (int stack : {32, 48, 64}) {
        if (st != NEB_OK) break;
        if (stack <= c->forest_depth) continue;
        int maxb = lds_blocks_per_cu(stack);
        for (int b : {0, 4, 8, 12, 16, maxb}) {
            if (b > maxb) continue;
            neb_launch_config cfg{stack, b, -1, best.photon_blocks_per_cu, best.photon_order, best.concurrent};
            double ms = 0.0;
            st = time_config(c, cfg, trial_iterations, trace_k, 2, s, ms);
            if (st != NEB_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best.bvh_stack = stack;
                best.trace_blocks_per_cu = b;
            }
        }
    }
    best_ms = 1e300;
    const int nee_k[1] = {K_NEE};
    for (int b : {0, 4, 8, 12, 16, lds_blocks_per_cu(best.bvh_stack)}) {
        if (st != NEB_OK) break;
        if (b > lds_blocks_per_cu(best.bvh_stack)) continue;
        neb_launch_config cfg{best.bvh_stack, best.trace_blocks_per_cu, b, best.photon_blocks_per_cu,
                              best.photon_order, best.concurrent};
        double ms = 0.0;
        st = time_config(c, cfg, trial_iterations, nee_k, 1, s, ms);
        if (st != NEB_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best.nee_blocks_per_cu = b;
        }
    }
    best_ms = 1e300;
    // the photon stage: ordering (which also adds to the photon traversal) and the merge grid
    const int photon_k[4] = {K_PHOTON, K_PHOTON_ORDER, K_EXTEND_PHOTON, K_PHOTON_SCATTER};
    for (int order : {1, 0}) {
        for (int pb : {0, 8, 16, 32, 64}) {
            if (st != NEB_OK) break;
            neb_launch_config cfg{best.bvh_stack, best.trace_blocks_per_cu, best.nee_blocks_per_cu, pb, order,
                                  best.concurrent};
            double ms = 0.0;
            st = time_config(c, cfg, trial_iterations, photon_k, 4, s, ms);
            if (st != NEB_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best.photon_blocks_per_cu = pb;
                best.photon_order = order;
            }
        }
    }
    prof_clear(c);
    c->prof_on = false;
    if (st == NEB_OK) {
        const neb_launch_config base = best;
        const int maxb = lds_blocks_per_cu(base.bvh_stack);
        best_ms = 1e300;
        for (int order : {base.photon_order, 1 - base.photon_order})
            for (int tb : {base.trace_blocks_per_cu, 8, 10, 12, 16}) {
                for (int pb : {base.photon_blocks_per_cu, 16, 24, 32}) {
                    if (st != NEB_OK) break;
                    if (tb > maxb) continue;
                    neb_launch_config cfg = base;
                    cfg.photon_order = order;
                    cfg.trace_blocks_per_cu = tb;
                    cfg.photon_blocks_per_cu = pb;
                    double ms = 0.0;
                    st = time_iterations(c, cfg, trial_iterations, s, ms);
                    if (st != NEB_OK) break;
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = cfg;
                    }
                }
            }
    }
    c->prof_on = was_on;
    if (st != NEB_OK) {
        c->cfg = keep;
        drop_graph(c);
        return st;
    }
    st = apply_config(c, best);
    if (st != NEB_OK) return st;
    if (chosen) *chosen = best;
    return neb_reset(c);
}

extern "C" void neb_destroy(neb_ctx c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    destroy_ctx(c);
}

// ---------------------------------------------------------------------------
// learned density C ABI
// ---------------------------------------------------------------------------
static neb_status check_mlp_params(const neb_mlp_params& m) {
    if (m.train_iterations < 1 || m.train_iterations > 1000)
        return fail(NEB_ERR_INVALID_ARG, "train_iterations out of range (1..1000)");
    if (m.steps_per_iteration < 0 || m.steps_per_iteration > 100000)
        return fail(NEB_ERR_INVALID_ARG, "steps_per_iteration out of range (0..100000)");
    if (m.batch < 16 || m.batch > (1 << 20)) return fail(NEB_ERR_INVALID_ARG, "batch out of range (16..2^20)");
    if (!(m.lr > 0.f) || !(m.beta1 >= 0.f && m.beta1 < 1.f) || !(m.beta2 >= 0.f && m.beta2 < 1.f) || !(m.eps > 0.f) ||
        !std::isfinite(m.lr) || !std::isfinite(m.eps))
        return fail(NEB_ERR_INVALID_ARG, "Adam settings out of range");
    if (m.probe_every < 1 || m.probes < 1 || m.probes > (1 << 24))
        return fail(NEB_ERR_INVALID_ARG, "probe settings out of range");
    if (!(m.max_rel_error > 0.f) || !std::isfinite(m.max_rel_error))
        return fail(NEB_ERR_INVALID_ARG, "max_rel_error must be > 0");
    return NEB_OK;
}

extern "C" neb_status neb_configure_mlp(neb_ctx c, const neb_mlp_params* params) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (!c->mlp_mode) return fail(NEB_ERR_STATE, "context was not created with NEB_DENSITY_MLP");
    neb_mlp_params m;
    if (params) m = *params;
    else mlp_defaults(m);
    neb_status st = check_mlp_params(m);
    if (st != NEB_OK) return st;
    HIP_TRY(hipDeviceSynchronize());
    if (m.batch > c->mlp.max_batch) {
        mlp_free(c->mlp);
        hipError_t e = mlp_alloc(c->mlp, m.batch);
        if (e != hipSuccess) {
            mlp_free(c->mlp);
            (void)mlp_alloc(c->mlp, c->mcfg.batch);
            return oom_or_device(e, "neb_configure_mlp");
        }
    }
    c->mcfg = m;
    if (c->ready) return neb_reset(c);
    return NEB_OK;
}

extern "C" neb_status neb_set_mlp_model(neb_ctx c, const float* params, float mu, float sigma) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (!c->mlp_mode) return fail(NEB_ERR_STATE, "context was not created with NEB_DENSITY_MLP");
    if (!params) {
        c->mlp_given = false;
        c->mlp_init.clear();
    } else {
        if (!std::isfinite(mu) || !(sigma > 0.f) || !std::isfinite(sigma))
            return fail(NEB_ERR_INVALID_ARG, "mu must be finite and sigma > 0");
        for (int i = 0; i < kMlpParams; ++i)
            if (!std::isfinite(params[i])) return fail(NEB_ERR_INVALID_ARG, "non-finite model parameter");
        c->mlp_init.assign(params, params + kMlpParams);
        c->mlp_mu = mu;
        c->mlp_sigma = sigma;
        c->mlp_given = true;
    }
    if (c->ready) return neb_reset(c);
    return NEB_OK;
}

extern "C" neb_status neb_get_mlp_gates(neb_ctx c, int32_t* gate, int32_t* probes, int32_t* bad) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (!c->mlp_mode) return fail(NEB_ERR_STATE, "context was not created with NEB_DENSITY_MLP");
    if (!c->ready) return fail(NEB_ERR_STATE, "scene not set");
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    if (gate) HIP_TRY(hipMemcpy(gate, c->reg_gate, 4 * (size_t)kRegions, hipMemcpyDeviceToHost));
    if (probes) HIP_TRY(hipMemcpy(probes, c->reg_total, 4 * (size_t)kRegions, hipMemcpyDeviceToHost));
    if (bad) HIP_TRY(hipMemcpy(bad, c->reg_bad, 4 * (size_t)kRegions, hipMemcpyDeviceToHost));
    return NEB_OK;
}

extern "C" neb_status neb_get_mlp_status(neb_ctx c, neb_mlp_status* out) {
    if (!c || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (!c->mlp_mode) return fail(NEB_ERR_STATE, "context was not created with NEB_DENSITY_MLP");
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    unsigned long long mc[kMlpCnt];
    MlpNorm nm;
    float loss = 0.f;
    HIP_TRY(hipMemcpy(mc, c->mlp_cnt, sizeof(mc), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&nm, c->mlp.norm, sizeof(nm), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&loss, c->mlp.loss, sizeof(loss), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->phase = c->iter > c->mcfg.train_iterations ? 1 : 0;
    out->adam_steps = c->mlp.step;
    double denom = (double)c->last_train_steps * (double)c->mcfg.batch;
    out->last_loss = denom > 0 ? (double)loss / denom : 0.0;
    out->mu = nm.mu;
    out->sigma = nm.sigma;
    out->probes = (int64_t)mc[kMlpCntProbes];
    out->probes_bad = (int64_t)mc[kMlpCntBad];
    out->regions_probed = (int64_t)mc[kMlpCntProbed];
    out->regions_disabled = (int64_t)mc[kMlpCntDisabled];
    out->fallback_queries = (int64_t)mc[kMlpCntFallback];
    out->probes_served = (int64_t)mc[kMlpCntServed];
    out->probes_served_bad = (int64_t)mc[kMlpCntServedBad];
    return NEB_OK;
}

extern "C" neb_status neb_get_mlp_weights(neb_ctx c, float* params) {
    if (!c || !params) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (!c->mlp_mode) return fail(NEB_ERR_STATE, "context was not created with NEB_DENSITY_MLP");
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    HIP_TRY(hipMemcpy(params, c->mlp.theta, 4 * (size_t)kMlpParams, hipMemcpyDeviceToHost));
    return NEB_OK;
}

struct neb_mlp_s {
    Mlp m;
};

extern "C" neb_status neb_mlp_create(const float* init, uint32_t seed, int32_t max_batch, neb_mlp* out) {
    if (!out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 20)) return fail(NEB_ERR_INVALID_ARG, "max_batch out of range (1..2^20)");
    std::vector<float> w;
    if (init) {
        w.assign(init, init + kMlpParams);
        for (float x : w)
            if (!std::isfinite(x)) return fail(NEB_ERR_INVALID_ARG, "non-finite initial parameter");
    } else {
        w = mlp_he_init(seed);
    }
    neb_mlp h = new neb_mlp_s();
    hipError_t e = mlp_alloc(h->m, max_batch);
    if (e == hipSuccess) e = mlp_set_weights(h->m, w.data(), nullptr);
    if (e == hipSuccess) e = mlp_set_norm(h->m, 0.f, 1.f, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        mlp_free(h->m);
        delete h;
        return oom_or_device(e, "neb_mlp_create");
    }
    *out = h;
    return NEB_OK;
}

extern "C" neb_status neb_mlp_set_normalization(neb_mlp h, float mu, float sigma, void* stream) {
    if (!h) return fail(NEB_ERR_INVALID_ARG, "null model");
    if (!std::isfinite(mu) || !(sigma > 0.f) || !std::isfinite(sigma))
        return fail(NEB_ERR_INVALID_ARG, "mu must be finite and sigma > 0");
    HIP_TRY(mlp_set_norm(h->m, mu, sigma, (hipStream_t)stream));
    return NEB_OK;
}

extern "C" neb_status neb_mlp_infer(neb_mlp h, const float* q, const float* nrm, int32_t n, float* out, void* stream) {
    if (!h || ((!q || !nrm || !out) && n > 0)) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (n < 0) return fail(NEB_ERR_INVALID_ARG, "negative count");
    HIP_TRY(mlp_infer(h->m, q, 3, nrm, 3, nullptr, n, nullptr, out, 0, (hipStream_t)stream));
    return NEB_OK;
}

static neb_status mlp_batch_grad(neb_mlp h, const float* q, const float* nrm, const float* t, int32_t n,
                                 hipStream_t s) {
    if (!h || !q || !nrm || !t) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (n < 1 || n > h->m.max_batch) return fail(NEB_ERR_INVALID_ARG, "batch size out of range (1..max_batch)");
    HIP_TRY(hipMemsetAsync(h->m.loss, 0, sizeof(float), s));
    HIP_TRY(mlp_gradient(h->m, q, 3, nrm, 3, t, nullptr, n, n, 0, 0u, 0u, nullptr, s));
    return NEB_OK;
}

extern "C" neb_status neb_mlp_gradient(neb_mlp h, const float* q, const float* nrm, const float* log_rho, int32_t n,
                                       float* grad, float* loss, void* stream) {
    if (!grad || !loss) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    neb_status st = mlp_batch_grad(h, q, nrm, log_rho, n, s);
    if (st != NEB_OK) return st;
    HIP_TRY(hipMemcpyAsync(grad, h->m.grad, 4 * (size_t)kMlpParams, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(h->m.grad, 0, 4 * (size_t)kMlpParams, s));
    float sum = 0.f;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(&sum, h->m.loss, sizeof(float), hipMemcpyDeviceToHost));
    *loss = sum / (float)n;
    return NEB_OK;
}

extern "C" neb_status neb_mlp_train_step(neb_mlp h, const float* q, const float* nrm, const float* log_rho, int32_t n,
                                         float lr, float beta1, float beta2, float eps, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(NEB_ERR_INVALID_ARG, "Adam settings out of range");
    neb_status st = mlp_batch_grad(h, q, nrm, log_rho, n, s);
    if (st != NEB_OK) return st;
    HIP_TRY(mlp_adam(h->m, lr, beta1, beta2, eps, s));
    return NEB_OK;
}

extern "C" neb_status neb_mlp_get_params(neb_mlp h, float* params) {
    if (!h || !params) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(params, h->m.theta, 4 * (size_t)kMlpParams, hipMemcpyDeviceToHost));
    return NEB_OK;
}

extern "C" void neb_mlp_destroy(neb_mlp h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    mlp_free(h->m);
    delete h;
}

// ---------------------------------------------------------------------------
// octree C ABI
// ---------------------------------------------------------------------------
extern "C" neb_status neb_octree_create(const float scene_min[3], const float scene_max[3], int32_t capacity,
                                        neb_octree* out) {
    if (!scene_min || !scene_max || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    if (capacity < 1 || capacity > (1 << 29)) return fail(NEB_ERR_INVALID_ARG, "capacity out of range");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(scene_min[k]) || !std::isfinite(scene_max[k]) || !(scene_max[k] > scene_min[k]))
            return fail(NEB_ERR_INVALID_ARG, "bounds must be finite with max > min");
    neb_octree o = new neb_octree_s();
    Octree& t = o->o;
    octree_params_init(t.prm, scene_min, scene_max, 0, capacity);
    t.capacity = t.prm.end;
    t.last_iter = 1;
    hipError_t e = hipMalloc(&t.nodes, 4 * (size_t)t.capacity);
    if (e == hipSuccess) e = hipMalloc(&t.state, sizeof(OctState));
    if (e == hipSuccess) e = hipMalloc(&t.dyn, sizeof(OctDyn));
    if (e == hipSuccess) e = hipMalloc(&t.prm_dev, sizeof(OctParams));
    if (e == hipSuccess) e = hipMemcpy(t.prm_dev, &t.prm, sizeof(OctParams), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = octree_reset(t, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        octree_release(t);
        delete o;
        return oom_or_device(e, "neb_octree_create");
    }
    *out = o;
    return NEB_OK;
}

extern "C" neb_status neb_octree_set_iteration(neb_octree o, int32_t iter) {
    if (!o) return fail(NEB_ERR_INVALID_ARG, "null octree");
    if (iter < 1) return fail(NEB_ERR_INVALID_ARG, "iteration must be >= 1");
    if (iter < o->o.last_iter) return fail(NEB_ERR_STATE, "iterations must not decrease");
    OctDyn d;
    octree_dyn_for(d, iter);
    // the scalars live in device memory: wait for every launch that may read
    // them, then write them synchronously
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(o->o.dyn, &d, sizeof(d), hipMemcpyHostToDevice));
    o->o.last_iter = iter;
    return NEB_OK;
}

extern "C" neb_status neb_octree_increment(neb_octree o, const float* pos, int32_t n, int32_t single, void* stream) {
    if (!o || (!pos && n > 0)) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (n < 0) return fail(NEB_ERR_INVALID_ARG, "negative count");
    HIP_TRY(octree_increment_xyz(o->o, pos, n, single, (hipStream_t)stream));
    return NEB_OK;
}

extern "C" neb_status neb_octree_density(neb_octree o, const float* pos, const float* nrm, int32_t n, int32_t robust,
                                         float* out, void* stream) {
    if (!o || ((!pos || !nrm || !out) && n > 0)) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (n < 0) return fail(NEB_ERR_INVALID_ARG, "negative count");
    HIP_TRY(octree_density_xyz(o->o, pos, nrm, n, robust, out, (hipStream_t)stream));
    return NEB_OK;
}

extern "C" neb_status neb_octree_clear_counters(neb_octree o, void* stream) {
    if (!o) return fail(NEB_ERR_INVALID_ARG, "null octree");
    HIP_TRY(octree_clear(o->o, (hipStream_t)stream));
    o->o.last_iter = 1;
    return NEB_OK;
}

extern "C" neb_status neb_octree_export(neb_octree o, int32_t* nodes, int32_t cap, int64_t info[8], void* stream) {
    if (!o || !info) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    neb_status st = octree_info(o->o.nodes, o->o.state, 0, o->o.capacity, (hipStream_t)stream, info);
    if (st != NEB_OK) return st;
    if (nodes && cap > 0)
        HIP_TRY(hipMemcpy(nodes, o->o.nodes, 4 * (size_t)std::min(cap, o->o.capacity), hipMemcpyDeviceToHost));
    return NEB_OK;
}

extern "C" void neb_octree_destroy(neb_octree o) {
    if (!o) return;
    (void)hipDeviceSynchronize();
    octree_release(o->o);
    delete o;
}
