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
//   pass 3  emitter-hit events weighted with w_e (Sec. 3.3)
// MIS weights (Sec. 4, balance heuristic over e, E and P_k) are evaluated
// with running ratios carried by the view and photon states, so no event
// needs the full path: each view vertex stores B = A_{m-2} + [x_{m-1} not
// delta] and g = |cos out at x_{m-1}| / (pdf at x_{m-1} * |cos in at x_m|),
// each photon carries U and h with the same meaning from the light side.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "neb_bvh.h"
#include "neb_device.h"

namespace neb {

// ---------------------------------------------------------------------------
// state layouts (SoA of float4, ints stored as float bits)
//   path q0 (o.xyz, pixel)  q1 (d.xyz, depth of the next hit)
//        q2 (tau.rgb, pdf of the sampled direction at the last vertex)
//        q3 (A_{m-1}, |cos out|/pdf at the last vertex, last vertex non-delta, last vertex index)
//   vertex v0 (pos, pixel)  v1 (n, depth | material << 8)  v2 (wo, B)  v3 (tau, g)
//   event e0 (tau*Le, p_light/f or 0 for a direct hit)  e1 (A, prev non-delta, prev vertex, pixel)
//   photon p0 (o, origin pixel)  p1 (d, 16*origin depth + bounce)  p2 (Phi, |cos out|/pdf)  pu (U)
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
};
struct Images {
    float *e, *E, *P;
};
// Merge grid keyed by (cell hash, depth - 1): the records of one cell are
// ordered by view-vertex depth, so the vertices a photon after j bounces may
// merge with (depth <= maxlen - 1 - j) form one contiguous prefix.
struct Grid {
    int32_t* count;   // T * D + 1 entries (the last stays 0)
    int32_t* start;   // T * D + 1 entries
    float4* sorted;   // (pos, vertex index) in (cell, depth) order
    float4* mrec;     // 4 per record, same order: what a merge needs of the view vertex:
                      // (n, depth | material << 8), (wo, B), (tau, g), (pixel, -, -, -)
    int32_t* sums;    // scan block sums, all levels
    int32_t T;        // hash buckets (power of two)
    int32_t D;        // depth classes = maxlen - 1
    float inv_cell;
};

struct RenderArgs {
    SceneView S;
    CamParams cam;
    uint32_t k0, k1;
    int32_t iter;
    int32_t L;
    int32_t npix;
    int32_t photons;     // n_P > 0
    float r, r2pi;
    int32_t density_mode;
    float rho0, cam_w;
};

__device__ __forceinline__ int fbits(float f) { return __float_as_int(f); }
__device__ __forceinline__ float ibits(int i) { return __int_as_float(i); }

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
__global__ void k_iter_begin(Counters* c, int32_t npix) {
    c->qcount[0] = npix;
    c->qcount[1] = 0;
    c->pcount[0] = 0;
    c->pcount[1] = 0;
    c->n_vertices = 0;
    c->n_events = 0;
    c->paths += (unsigned long long)npix;
}
__global__ void k_iter_end(Counters* c) {
    c->vertices += (unsigned long long)c->n_vertices;
    c->events += (unsigned long long)c->n_events;
}
__global__ void k_mean_image(const float* e, const float* E, const float* P, float* out, int64_t n, float scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (e[i] + E[i] + P[i]) * scale;
}
__global__ void k_scale_image(const float* a, float* out, int64_t n, float scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] * scale;
}

// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_camera(RenderArgs A, PathQ q) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < A.npix; i += gridDim.x * blockDim.x) {
        int px = i % A.cam.w, py = i / A.cam.w;
        U4 u = uniforms(A.k0, A.k1, (uint32_t)i, (uint32_t)A.iter, 0u, kTagCamera);
        f3 d = cam_ray(A.cam, px, py, u.u[0], u.u[1]);
        q.q0[i] = f4(load3(A.cam.eye), ibits(i));
        q.q1[i] = f4(d, ibits(1));
        q.q2[i] = make_float4(1.f, 1.f, 1.f, 0.f);
        q.q3[i] = make_float4(0.f, 0.f, 0.f, ibits(-1));
    }
}

// closest hit for a queue of rays given as (origin, direction) float4 arrays;
// also clears the counter of the queue the next kernel appends to
__global__ void __launch_bounds__(kTraceBlock) k_extend(SceneView S, const float4* __restrict__ org,
                                                        const float4* __restrict__ dir, const int32_t* count,
                                                        int32_t* next_count, int2* __restrict__ hits,
                                                        unsigned long long* rays, Counters* cnt) {
    __shared__ int stack[kBvhStack * kTraceBlock];
    int n = *count;
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_count = 0;
    unsigned traced = 0, nodes = 0, tris = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float t;
        int prim = trace<false>(S, xyz(org[i]), xyz(dir[i]), INFINITY, t, stack + threadIdx.x, nodes, tris);
        hits[i] = make_int2(fbits(t), prim);
        ++traced;
    }
    wave_add_u64(rays, traced);
    wave_add_u64(&cnt->bvh_nodes, nodes);
    wave_add_u64(&cnt->bvh_tris, tris);
}

__global__ void __launch_bounds__(256) k_shade(RenderArgs A, PathQ in, const int32_t* count_in, const int2* hits,
                                               PathQ out, int32_t* count_out, VertexStore V, int32_t* n_vertices,
                                               float4* ev0, float4* ev1, int32_t* n_events, int32_t* slots,
                                               neb_path_record* rec) {
    int n = *count_in;
    const SceneView& S = A.S;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float4 a0 = in.q0[i], a1 = in.q1[i], a2 = in.q2[i], a3 = in.q3[i];
        int2 h = hits[i];
        int pixel = fbits(a0.w), k = fbits(a1.w);
        neb_path_record* rc = rec ? rec + (size_t)pixel * A.L + (k - 1) : nullptr;
        bool alive = h.y >= 0;
        if (!alive && rc) {
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
        bool emit = alive && mat_emits(m) && cin > 0.f && S.prim_light[prim] >= 0;
        int eslot = wave_reserve(n_events, emit);
        if (emit) {
            float q = 0.f;
            if (k > 1) {
                int lid = S.prim_light[prim];
                float p_light = S.lights[5 * lid].w / S.lights[5 * lid + 1].w;
                float f_prev = a2.w * cin / (t * t);
                q = p_light / f_prev;
            }
            ev0[eslot] = f4(tau * load3(m.emission), q);
            ev1[eslot] = make_float4(a3.x, a3.z, a3.w, ibits(pixel));
        }
        bool store = alive && !mat_black(m) && k <= A.L - 1;
        float g = (k >= 2) ? a3.y / fabsf(cin) : 0.f;
        float B = (k >= 2) ? a3.x + a3.z : 0.f;
        int vid = wave_reserve(n_vertices, store);
        if (store) {
            V.v0[vid] = f4(x, ibits(pixel));
            V.v1[vid] = f4(nrm, ibits(k | (mid << 8)));
            V.v2[vid] = f4(wo, B);
            V.v3[vid] = f4(tau, g);
            if (slots) slots[(size_t)(k - 1) * A.npix + pixel] = vid;
        }
        Sample s;
        s.ev = 0;
        if (store) {
            U4 u = uniforms(A.k0, A.k1, (uint32_t)pixel, (uint32_t)A.iter, (uint32_t)k, kTagBsdf);
            s = bsdf_sample(m, nrm, wo, u);
        }
        bool go = s.ev != 0;
        if (go && rc) rc->type = s.ev;
        int slot = wave_reserve(count_out, go);
        if (go) {
            float Acur = (k >= 2) ? bsdf_pdf(m, nrm, s.dir, wo) * g * B : 0.f;
            float gp = fabsf(dot3(nrm, s.dir)) / s.pdf;
            float dnon = mat_delta(m.type) ? 0.f : 1.f;
            out.q0[slot] = f4(offset_origin(x, nrm, s.dir, S.eps), ibits(pixel));
            out.q1[slot] = f4(s.dir, ibits(k + 1));
            out.q2[slot] = f4(tau * s.w, s.pdf);
            out.q3[slot] = make_float4(Acur, gp, dnon, ibits(vid));
        }
    }
}

// ---------------------------------------------------------------------------
// pass 2 (a): density at every NEE vertex
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_density(RenderArgs A, VertexStore V, const int32_t* n_vertices,
                                                 const int32_t* __restrict__ nodes, const OctState* ost,
                                                 OctParams P) {
    int n = *n_vertices;
    int depth = ost->depth;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        f3 x = xyz(V.v0[i]), nn = xyz(V.v1[i]);
        float rho;
        if (A.density_mode == NEB_DENSITY_ANALYTIC)
            rho = A.rho0 + A.cam_w * cam_hit_density(A.cam, x, nn);
        else if (A.density_mode == NEB_DENSITY_OCTREE)
            rho = oct_query(nodes, P, depth, x, nn, false, nullptr);
        else
            rho = oct_query_robust(nodes, P, depth, x, nn);
        V.rho[i] = rho;
    }
}

// ---------------------------------------------------------------------------
// pass 2 (b, c): NEE and the photon that reuses its segment
// ---------------------------------------------------------------------------
struct LightSample {
    f3 x, n, w, dE;
    float d2, cos_l, p_light;
    bool hittable;
};

__device__ __forceinline__ LightSample sample_light(const SceneView& S, f3 x, f3 nx, const U4& u) {
    LightSample ls;
    ls.dE = mk3(0.f, 0.f, 0.f);
    ls.hittable = false;
    ls.p_light = 0.f;
    ls.cos_l = 0.f;
    int lo = 0, hi = S.n_lights - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (u.u[0] < S.light_cdf[mid]) hi = mid;
        else lo = mid + 1;
    }
    const float4* L = S.lights + 5 * lo;
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

__global__ void __launch_bounds__(kTraceBlock) k_nee(RenderArgs A, VertexStore V, const int32_t* n_vertices,
                                                     Images img, PhotonQ pq, int32_t* pcount, Counters* cnt) {
    __shared__ int stack[kBvhStack * kTraceBlock];
    int n = *n_vertices;
    const SceneView& S = A.S;
    unsigned vis = 0, emitted = 0, rays = 0, nodes = 0, tris = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float4 a0 = V.v0[i], a1 = V.v1[i], a2 = V.v2[i], a3 = V.v3[i];
        float rho = V.rho[i];
        f3 x = xyz(a0), nrm = xyz(a1), wo = xyz(a2), tau = xyz(a3);
        int pixel = fbits(a0.w);
        int packed = fbits(a1.w);
        int k = packed & 0xFF, mid = packed >> 8;
        const neb_material& m = S.mats[mid];
        U4 u = uniforms(A.k0, A.k1, (uint32_t)pixel, (uint32_t)A.iter, (uint32_t)k, kTagNee);
        LightSample ls = sample_light(S, x, nrm, u);
        bool ok = !is_zero3(ls.dE);
        if (ok) {
            f3 so = offset_origin(x, nrm, ls.w, S.eps);
            f3 sd = ls.x - so;
            float sl = sqrtf(dot3(sd, sd));
            float tt;
            ++rays;
            ok = trace<true>(S, so, sd * (1.0f / sl), (1.0f - 1e-5f) * sl, tt, stack + threadIdx.x, nodes, tris) < 0;
        }
        bool photon = false;
        Sample s;
        s.ev = 0;
        if (ok) {
            ++vis;
            bool dnon = !mat_delta(m.type);
            if (dnon) {
                f3 f = bsdf_f(m, nrm, wo, ls.w);
                if (!is_zero3(f)) {
                    float Am1 = (k >= 2) ? bsdf_pdf(m, nrm, ls.w, wo) * a3.w * a2.w : 0.f;
                    float ratio = 1.0f;
                    if (ls.hittable) ratio += bsdf_pdf(m, nrm, wo, ls.w) * ls.cos_l / (ls.d2 * ls.p_light);
                    if (A.photons) ratio += rho * A.r2pi * Am1;
                    atomic_add3(img.E, pixel, tau * f * ls.dE * (1.0f / ratio));
                }
            }
            if (A.photons && rho > 0.f) {
                U4 up = uniforms(A.k0, A.k1, (uint32_t)pixel, (uint32_t)A.iter, (uint32_t)(16 * k), kTagPhoton);
                s = bsdf_sample(m, nrm, ls.w, up);
                photon = s.ev != 0;
            }
        }
        int slot = wave_reserve(pcount, photon);
        if (photon) {
            ++emitted;
            float fo = ls.hittable ? bsdf_pdf(m, nrm, s.dir, ls.w) * ls.cos_l / (ls.d2 * ls.p_light) : 0.f;
            float dnon = mat_delta(m.type) ? 0.f : 1.f;
            float U1 = (fo + dnon) / (rho * A.r2pi);
            float hp = fabsf(dot3(nrm, s.dir)) / s.pdf;
            f3 phi = ls.dE * (1.0f / rho) * s.w;
            pq.p0[slot] = f4(offset_origin(x, nrm, s.dir, S.eps), ibits(pixel));
            pq.p1[slot] = f4(s.dir, ibits(16 * k + 1));
            pq.p2[slot] = f4(phi, hp);
            pq.pu[slot] = U1;
        }
    }
    wave_add_u64(&cnt->nee_visible, vis);
    wave_add_u64(&cnt->photons, emitted);
    wave_add_u64(&cnt->shadow_rays, rays);
    wave_add_u64(&cnt->bvh_nodes, nodes);
    wave_add_u64(&cnt->bvh_tris, tris);
}

// ---------------------------------------------------------------------------
// merge structure: hash grid of cell size 2r over the non-delta view vertices
// (count -> exclusive scan -> scatter); count[] returns to zero after scatter
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cell_hash(int cx, int cy, int cz, int32_t T) {
    return (((uint32_t)cx * 73856093u) ^ ((uint32_t)cy * 19349663u) ^ ((uint32_t)cz * 83492791u)) & (uint32_t)(T - 1);
}
__device__ __forceinline__ uint32_t point_hash(f3 p, float inv_cell, int32_t T) {
    return cell_hash((int)floorf(p.x * inv_cell), (int)floorf(p.y * inv_cell), (int)floorf(p.z * inv_cell), T);
}

__device__ __forceinline__ int64_t grid_key(const Grid& G, uint32_t h, int depth) {
    return (int64_t)h * G.D + (depth - 1);
}

__global__ void __launch_bounds__(256) k_grid_count(const neb_material* mats, VertexStore V, const int32_t* n_vertices,
                                                    Grid G) {
    int n = *n_vertices;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int packed = fbits(V.v1[i].w);
        if (mat_delta(mats[packed >> 8].type)) continue;
        atomicAdd(&G.count[grid_key(G, point_hash(xyz(V.v0[i]), G.inv_cell, G.T), packed & 0xFF)], 1);
    }
}

__global__ void __launch_bounds__(256) k_grid_scatter(const neb_material* mats, VertexStore V,
                                                      const int32_t* n_vertices, Grid G) {
    int n = *n_vertices;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int packed = fbits(V.v1[i].w);
        if (mat_delta(mats[packed >> 8].type)) continue;
        f3 p = xyz(V.v0[i]);
        int64_t key = grid_key(G, point_hash(p, G.inv_cell, G.T), packed & 0xFF);
        int pos = G.start[key] + atomicSub(&G.count[key], 1) - 1;
        G.sorted[pos] = f4(p, ibits(i));
        float4* m = G.mrec + 4 * (size_t)pos;
        m[0] = V.v1[i];
        m[1] = V.v2[i];
        m[2] = V.v3[i];
        m[3] = make_float4(V.v0[i].w, 0.f, 0.f, 0.f);
    }
}

// exclusive scan in three launches: 4096 elements per block of 256 threads
constexpr int kScanPer = 16;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanPer * kScanBlock;

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

__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(const int32_t* in, int32_t* out, int32_t* sums, int64_t n) {
    __shared__ int sh[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int loc[kScanPer];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        loc[k] = (base + k < n) ? in[base + k] : 0;
        s += loc[k];
    }
    int total;
    int pre = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = pre;
        pre += loc[k];
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
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) out[base + k] += add;
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

// exclusive prefix sum of n ints (in and out may alias): tiles of 4096,
// then the tile sums recursively, then the offsets added back
static void scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch, hipStream_t s) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, scratch, n);
    if (nb <= kScanTile) {
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, scratch, (int32_t)nb);
    } else {
        scan_exclusive(scratch, scratch, nb, scratch + nb, s);
    }
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, out, scratch, n);
}

// ---------------------------------------------------------------------------
// photon bounce: merge with view vertices around the hit, then scatter.
// One photon per lane (many independent candidate streams in flight, which
// is what a gather over cache-resident records needs).  Each lane walks the
// concatenated candidate ranges of its photon's cells; accepted (lane,
// vertex) pairs are compacted into an LDS queue and evaluated 64 at a time
// by the whole wave, so the BSDF, the MIS weight and the image atomics run
// with every lane busy instead of with the ~10 % of lanes that accepted.
// One wave per block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_photon(RenderArgs A, PhotonQ in, const int32_t* count_in, const int2* hits,
                                               PhotonQ out, int32_t* count_out, VertexStore V, Grid G, Images img,
                                               Counters* cnt) {
    __shared__ int2 queue[128];
    __shared__ float4 tp[64][2];  // per lane's photon: (-d, h*U), (Phi / (pi r^2), bounce)
    const int lane = threadIdx.x;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int n = *count_in;
    const SceneView& S = A.S;
    unsigned segs = 0, merges = 0, items = 0, cont = 0, cells = 0, cands = 0;
    const float r2 = A.r * A.r;
    const float kern = 1.0f / A.r2pi;
    const float cell = 1.0f / G.inv_cell;
    int qn = 0;  // queue length, identical in every lane

    auto flush = [&](int count) {
        if (lane < count) {
            int2 pr = queue[lane];
            float4 t0 = tp[pr.x][0], t1 = tp[pr.x][1];
            const float4* mr = G.mrec + 4 * (size_t)pr.y;  // one 64-byte record
            float4 v1 = mr[0];
            int packed = fbits(v1.w);
            int k = packed & 0xFF;
            if (k + fbits(t1.w) + 1 <= A.L) {
                const neb_material& mv = S.mats[packed >> 8];
                float4 v2 = mr[1];
                f3 nv = xyz(v1), wv = xyz(v2), wd = xyz(t0);
                f3 f = bsdf_f(mv, nv, wv, wd);
                if (!is_zero3(f)) {
                    float4 v3 = mr[2];
                    float T = bsdf_pdf(mv, nv, wv, wd) * t0.w;
                    float C = 1.0f + ((k >= 2) ? bsdf_pdf(mv, nv, wd, wv) * v3.w * v2.w : 0.f);
                    int vpix = fbits(mr[3].x);
                    atomic_add3(img.P, vpix, xyz(v3) * f * xyz(t1) * (1.0f / (C + T)));
                    ++merges;
                }
            }
        }
    };

    for (int base = blockIdx.x * 64; base < n; base += gridDim.x * 64) {
        int i = base + lane;
        bool valid = i < n;
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
        int code = fbits(b1.w);
        int j = code & 15, odepth = code >> 4, opix = fbits(b0.w);
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
        tp[lane][0] = f4(-d, hh * U);
        tp[lane][1] = f4(xyz(b2) * kern, ibits(j));
        // candidate ranges of the (at most 8) cells the ball touches
        int lo[8], pre[9];
        pre[0] = 0;
        const int kmax = A.L - 1 - j;  // deepest view vertex this photon may merge with
        {
            float rr = A.r * 1.00001f;
            int lx = (int)floorf((y.x - rr) * G.inv_cell), hx = min((int)floorf((y.x + rr) * G.inv_cell), lx + 1);
            int ly = (int)floorf((y.y - rr) * G.inv_cell), hy = min((int)floorf((y.y + rr) * G.inv_cell), ly + 1);
            int lz = (int)floorf((y.z - rr) * G.inv_cell), hz = min((int)floorf((y.z + rr) * G.inv_cell), lz + 1);
            uint32_t seen[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                int cx = lx + (c & 1), cy = ly + ((c >> 1) & 1), cz = lz + ((c >> 2) & 1);
                bool use = mergeable && cx <= hx && cy <= hy && cz <= hz;
                // skip cells whose box is farther than r from the hit
                float dx = fmaxf(fmaxf(cx * cell - y.x, y.x - (cx + 1) * cell), 0.f);
                float dy = fmaxf(fmaxf(cy * cell - y.y, y.y - (cy + 1) * cell), 0.f);
                float dz = fmaxf(fmaxf(cz * cell - y.z, y.z - (cz + 1) * cell), 0.f);
                use = use && dx * dx + dy * dy + dz * dz <= r2 * 1.0001f;
                uint32_t hc = cell_hash(cx, cy, cz, G.T);
                seen[c] = use ? hc : 0xFFFFFFFFu;
#pragma unroll
                for (int q = 0; q < c; ++q) use = use && seen[q] != hc;
                int e0 = 0, e1 = 0;
                if (use) {
                    int64_t key = grid_key(G, hc, 1);
                    e0 = G.start[key];
                    e1 = G.start[key + kmax];
                    ++cells;
                }
                lo[c] = e0;
                pre[c + 1] = pre[c] + (e1 - e0);
            }
        }
        int total = pre[8];
        cands += (unsigned)total;
        __syncthreads();
        for (int k = 0;; ++k) {
            bool act = k < total;
            if (!__any(act)) break;
            bool acc = false;
            int vid = 0;
            if (act) {
                int e = 0;
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (k >= pre[c] && k < pre[c + 1]) e = lo[c] + (k - pre[c]);
                float4 cd = G.sorted[e];
                f3 dv = xyz(cd) - y;
                acc = dot3(dv, dv) < r2;
                vid = e;  // the record index: its merge data sits at G.mrec[4 e]
            }
            unsigned long long m = __ballot(acc);
            if (m) {
                if (acc) queue[qn + __popcll(m & below)] = make_int2(lane, vid);
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
        if (qn > 0) {
            __syncthreads();
            flush(qn);
            qn = 0;
        }
        // scatter
        bool go = false;
        Sample s;
        s.ev = 0;
        if (hit && j < A.L - 2 && !mat_black(my)) {
            U4 u = uniforms(A.k0, A.k1, (uint32_t)opix, (uint32_t)A.iter, (uint32_t)(16 * odepth + j), kTagPhoton);
            s = bsdf_sample(my, ny, -d, u);
            go = s.ev != 0;
        }
        int slot = wave_reserve(count_out, go);
        cont += go;
        if (go) {
            f3 wd = -d;
            float prev = bsdf_pdf(my, ny, s.dir, wd);
            float Un = (mat_delta(my.type) ? 0.f : 1.f) + prev * hh * U;
            float hp = fabsf(dot3(ny, s.dir)) / s.pdf;
            out.p0[slot] = f4(offset_origin(y, ny, s.dir, S.eps), ibits(opix));
            out.p1[slot] = f4(s.dir, ibits(16 * odepth + j + 1));
            out.p2[slot] = f4(xyz(b2) * s.w, hp);
            out.pu[slot] = Un;
        }
        __syncthreads();
    }
    wave_add_u64(&cnt->photon_segments, segs);
    wave_add_u64(&cnt->merges, merges);
    wave_add_u64(&cnt->photon_items, items);
    wave_add_u64(&cnt->photon_continued, cont);
    wave_add_u64(&cnt->grid_cells, cells);
    wave_add_u64(&cnt->candidates, cands);
}

// ---------------------------------------------------------------------------
// pass 3: emitter hits
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_finalize(RenderArgs A, const float4* ev0, const float4* ev1,
                                                  const int32_t* n_events, const float* rho, Images img) {
    int n = *n_events;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float4 a = ev0[i], b = ev1[i];
        float w = 1.0f;
        if (a.w > 0.f) {
            int pv = fbits(b.z);
            float ratio = b.y;
            if (A.photons) ratio += rho[pv] * A.r2pi * b.x;
            w = 1.0f / (1.0f + a.w * ratio);
        }
        atomic_add3(img.e, fbits(b.w), xyz(a) * w);
    }
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

struct neb_ctx_s {
    neb_params prm{};
    int npix = 0, L = 0;
    int64_t vcap = 0, ecap = 0;
    // scene
    bool has_scene = false;
    float4 *bvh = nullptr, *tri = nullptr, *prim_n = nullptr, *lights = nullptr;
    int32_t* prim_light = nullptr;
    float* light_cdf = nullptr;
    neb_material* mats = nullptr;
    SceneView view{};
    CamParams cam{};
    Octree oct;
    // pools
    PathQ q[2]{};
    PhotonQ pq[2]{};
    int2* hits = nullptr;
    VertexStore V{};
    float4 *ev0 = nullptr, *ev1 = nullptr;
    int32_t* slots = nullptr;
    neb_path_record* recs = nullptr;
    Grid G{};
    float* img = nullptr;  // e, E, P accumulators
    Counters* cnt = nullptr;
    int32_t iter = 0;
    int32_t first_iter_recorded = 0;
    int32_t trace_grid = 4096;  // resident traversal blocks on this device
    hipStream_t last_stream = nullptr;
    std::vector<void*> allocs;
    std::vector<void*> scene_allocs;
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
    K_FINALIZE, K_MISC, K_COUNT
};
static const char* kKernelNames[K_COUNT] = {"camera", "extend_camera", "shade", "octree_insert", "density", "nee",
                                            "grid_build", "extend_photon", "photon_merge", "finalize", "misc"};

static void prof_harvest(neb_ctx c) {
    if (c->prof_used == 0) return;
    (void)hipEventSynchronize(c->prof_ev[c->prof_used - 1]);
    for (int i = 0; i < c->prof_used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->prof_ev[i], c->prof_ev[i + 1]) == hipSuccess) {
            c->prof_ms[c->prof_kid[i / 2]] += ms;
            c->prof_launches[c->prof_kid[i / 2]] += 1;
        }
    }
    c->prof_used = 0;
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

extern "C" neb_status neb_create(const neb_params* p, neb_ctx* out) {
    if (!p || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    if (p->width < 1 || p->height < 1 || p->width > 8192 || p->height > 8192)
        return fail(NEB_ERR_INVALID_ARG, "image size out of range");
    if (p->max_path_len < 1 || p->max_path_len > kMaxPathLen) return fail(NEB_ERR_INVALID_ARG, "max_path_len out of range");
    if (p->octree_capacity < 1 || p->octree_capacity > (1 << 29)) return fail(NEB_ERR_INVALID_ARG, "octree capacity out of range");
    if (!(p->merge_radius > 0.f) || !std::isfinite(p->merge_radius)) return fail(NEB_ERR_INVALID_ARG, "merge radius must be > 0");
    if (p->density_mode != NEB_DENSITY_OCTREE && p->density_mode != NEB_DENSITY_OCTREE_ROBUST &&
        p->density_mode != NEB_DENSITY_ANALYTIC)
        return fail(NEB_ERR_INVALID_ARG, "unknown density mode");
    if (!std::isfinite(p->analytic_rho0) || !std::isfinite(p->analytic_cam_weight))
        return fail(NEB_ERR_INVALID_ARG, "analytic density parameters must be finite");
    int64_t npix = (int64_t)p->width * p->height;
    int64_t vcap = npix * std::max(1, p->max_path_len - 1);
    if (vcap * 4 > (int64_t)INT32_MAX) return fail(NEB_ERR_CAPACITY, "image too large for the vertex pool");
    neb_ctx c = new neb_ctx_s();
    c->prm = *p;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            c->trace_grid = cus * kTraceBlocksPerCU;
    }
    c->npix = (int)npix;
    c->L = p->max_path_len;
    c->vcap = vcap;
    c->ecap = npix * p->max_path_len;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, n)                                   \
    if (e == hipSuccess) e = dalloc(c->allocs, &(ptr), (size_t)(n));
    for (int b = 0; b < 2; ++b) {
        ALLOC(c->q[b].q0, npix);
        ALLOC(c->q[b].q1, npix);
        ALLOC(c->q[b].q2, npix);
        ALLOC(c->q[b].q3, npix);
        ALLOC(c->pq[b].p0, vcap);
        ALLOC(c->pq[b].p1, vcap);
        ALLOC(c->pq[b].p2, vcap);
        ALLOC(c->pq[b].pu, vcap);
    }
    ALLOC(c->hits, std::max<int64_t>(npix, vcap));
    ALLOC(c->V.v0, vcap);
    ALLOC(c->V.v1, vcap);
    ALLOC(c->V.v2, vcap);
    ALLOC(c->V.v3, vcap);
    ALLOC(c->V.rho, vcap);
    ALLOC(c->ev0, c->ecap);
    ALLOC(c->ev1, c->ecap);
    if (p->flags & NEB_FLAG_SINGLE_THREAD_OCTREE) ALLOC(c->slots, vcap);
    if (p->flags & NEB_FLAG_RECORD_PATHS) ALLOC(c->recs, npix * p->max_path_len);
    c->G.D = std::max(1, p->max_path_len - 1);
    c->G.T = (int32_t)std::max<uint64_t>(1024, std::min<uint64_t>(next_pow2((uint64_t)vcap) / 2, 1u << 23));
    c->G.inv_cell = 1.0f / (2.0001f * p->merge_radius);  // a little wider than the ball's diameter
    int64_t gkeys = (int64_t)c->G.T * c->G.D + 1;
    ALLOC(c->G.count, gkeys);
    ALLOC(c->G.start, gkeys);
    ALLOC(c->G.sorted, vcap);
    ALLOC(c->G.mrec, 4 * vcap);
    ALLOC(c->G.sums, scan_scratch(gkeys));
    ALLOC(c->img, 9 * npix);
    ALLOC(c->cnt, 1);
    ALLOC(c->oct.nodes, 1 + ((p->octree_capacity + 7) & ~7));
    ALLOC(c->oct.state, 1);
#undef ALLOC
    if (e == hipSuccess) e = octree_reserve(c->oct, vcap);
    if (e != hipSuccess) {
        neb_status s = oom_or_device(e, "neb_create");
        free_list(c->allocs);
        c->oct.nodes = nullptr;
        c->oct.state = nullptr;
        octree_release(c->oct);
        delete c;
        return s;
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(gkeys, 256)), dim3(256), 0, nullptr, c->G.count, 0, gkeys);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(9 * npix, 256)), dim3(256), 0, nullptr, c->img, 0.f, 9 * npix);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, nullptr, (int32_t*)c->cnt, 0,
                       (int64_t)(sizeof(Counters) / 4));
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        neb_status s = oom_or_device(e, "neb_create init");
        free_list(c->allocs);
        c->oct.nodes = nullptr;
        c->oct.state = nullptr;
        octree_release(c->oct);
        delete c;
        return s;
    }
    *out = c;
    return NEB_OK;
}

static bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

extern "C" neb_status neb_set_scene(neb_ctx c, const float* vertices, int32_t nv, const int32_t* tris,
                                    const int32_t* tri_material, int32_t nt, const neb_material* materials, int32_t nm,
                                    const neb_point_light* point_lights, int32_t npl, const neb_camera* camera) {
    if (!c || !vertices || !tris || !tri_material || !materials || !camera) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (nv < 3 || nt < 1 || nm < 1 || npl < 0 || (npl > 0 && !point_lights))
        return fail(NEB_ERR_INVALID_ARG, "bad scene sizes");
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

    // BVH
    BvhHost bvh;
    if (!build_bvh(vertices, nv, tris, nt, bvh)) return fail(NEB_ERR_INVALID_ARG, "BVH build failed");
    if (bvh.max_depth >= kBvhStack) return fail(NEB_ERR_CAPACITY, "BVH deeper than the traversal stack");
    // per-prim normals and light table (emissive triangles, then point lights)
    std::vector<float> prim_n(4 * (size_t)nt);
    std::vector<int32_t> prim_light(nt, -1);
    std::vector<double> w;
    std::vector<float> lights;
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
        for (int k = 0; k < 3; ++k) prim_n[4 * t + k] = len > 0 ? (float)(cr[k] / len) : (k == 2 ? 1.f : 0.f);
        int32_t mid = tri_material[t];
        std::memcpy(&prim_n[4 * t + 3], &mid, 4);
        const neb_material& m = materials[mid];
        if (emis(m) > 0.0 && len > 0) {
            prim_light[t] = (int32_t)w.size();
            double area = 0.5 * len;
            w.push_back(M_PI * area * emis(m));
            float L0[20] = {a[0], a[1], a[2], 0.f,
                            (float)e1[0], (float)e1[1], (float)e1[2], (float)area,
                            (float)e2[0], (float)e2[1], (float)e2[2], 0.f,
                            m.emission[0], m.emission[1], m.emission[2], 0.f,
                            prim_n[4 * t], prim_n[4 * t + 1], prim_n[4 * t + 2], 0.f};
            lights.insert(lights.end(), L0, L0 + 20);
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
        lights.insert(lights.end(), L0, L0 + 20);
    }
    int nl = (int)w.size();
    if (nl == 0) return fail(NEB_ERR_INVALID_ARG, "scene has no lights");
    double tot = 0.0;
    for (double x : w) tot += x;
    if (!(tot > 0.0)) return fail(NEB_ERR_INVALID_ARG, "scene lights carry no power");
    std::vector<float> cdf(nl);
    double acc = 0.0;
    for (int i = 0; i < nl; ++i) {
        acc += w[i];
        cdf[i] = (float)(acc / tot);
        lights[20 * (size_t)i + 3] = (float)(w[i] / tot);
    }
    cdf[nl - 1] = 1.0f;

    // upload
    free_list(c->scene_allocs);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &c->bvh, 4 * (size_t)bvh.n_nodes);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &c->tri, 3 * (size_t)nt);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &c->prim_n, (size_t)nt);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &c->prim_light, (size_t)nt);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &c->mats, (size_t)nm);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &c->lights, 5 * (size_t)nl);
    if (e == hipSuccess) e = dalloc(c->scene_allocs, &c->light_cdf, (size_t)nl);
    if (e != hipSuccess) return oom_or_device(e, "scene upload");
    HIP_TRY(hipMemcpy(c->bvh, bvh.nodes.data(), bvh.nodes.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->tri, bvh.tris.data(), bvh.tris.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->prim_n, prim_n.data(), prim_n.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->prim_light, prim_light.data(), prim_light.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->mats, materials, sizeof(neb_material) * (size_t)nm, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->lights, lights.data(), lights.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->light_cdf, cdf.data(), cdf.size() * 4, hipMemcpyHostToDevice));
    c->view.bvh = c->bvh;
    c->view.tri = c->tri;
    c->view.prim_n = c->prim_n;
    c->view.prim_light = c->prim_light;
    c->view.mats = c->mats;
    c->view.lights = c->lights;
    c->view.light_cdf = c->light_cdf;
    c->view.n_lights = nl;
    float dg[3] = {bmax[0] - bmin[0], bmax[1] - bmin[1], bmax[2] - bmin[2]};
    c->view.eps = 1e-5f * std::sqrt(dg[0] * dg[0] + dg[1] * dg[1] + dg[2] * dg[2]);
    // camera
    CamParams& C = c->cam;
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
    C.aspect = (float)c->prm.width / (float)c->prm.height;
    C.w = c->prm.width;
    C.h = c->prm.height;
    // octree over the scene bounds
    octree_params_init(c->oct.prm, bmin, bmax, c->prm.octree_capacity);
    HIP_TRY(octree_init_nodes(c->oct, nullptr));
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(9 * (int64_t)c->npix, 256)), dim3(256), 0, nullptr, c->img, 0.f,
                       9 * (int64_t)c->npix);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, nullptr, (int32_t*)c->cnt, 0, (int64_t)(sizeof(Counters) / 4));
    HIP_TRY(hipDeviceSynchronize());
    c->iter = 0;
    c->first_iter_recorded = 0;
    c->has_scene = true;
    return NEB_OK;
}

static RenderArgs make_args(neb_ctx c) {
    RenderArgs A;
    A.S = c->view;
    A.cam = c->cam;
    A.k0 = c->prm.seed;
    A.k1 = c->prm.scene_id;
    A.iter = c->iter;
    A.L = c->L;
    A.npix = c->npix;
    A.photons = (c->prm.flags & NEB_FLAG_NO_PHOTONS) ? 0 : 1;
    A.r = c->prm.merge_radius;
    A.r2pi = (float)(M_PI * (double)c->prm.merge_radius * (double)c->prm.merge_radius);
    A.density_mode = c->prm.density_mode;
    A.rho0 = c->prm.analytic_rho0;
    A.cam_w = c->prm.analytic_cam_weight;
    return A;
}

static neb_status render_iteration(neb_ctx c, hipStream_t s) {
    c->iter += 1;
    octree_params_set_iteration(c->oct.prm, c->iter);
    RenderArgs A = make_args(c);
    const int npix = c->npix, L = c->L;
    const int64_t vcap = c->vcap;
    Counters* cnt = c->cnt;
    bool record = c->recs && c->first_iter_recorded == 0;
    hipLaunchKernelGGL(k_iter_begin, dim3(1), dim3(1), 0, s, cnt, npix);
    if (c->slots)
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(vcap, 256)), dim3(256), 0, s, c->slots, -1, vcap);
    if (record)
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of((int64_t)npix * L * 6, 256)), dim3(256), 0, s, (int32_t*)c->recs, 0,
                           (int64_t)npix * L * 6);
    TIMED(K_CAMERA, hipLaunchKernelGGL(k_camera, dim3(grid_of(npix, 256)), dim3(256), 0, s, A, c->q[0]));
    // pass 1
    for (int k = 1; k <= L; ++k) {
        int in = (k - 1) & 1, out = k & 1;
        TIMED(K_EXTEND_CAMERA,
              hipLaunchKernelGGL(k_extend, dim3(grid_of(npix, kTraceBlock, 1 << 20)), dim3(kTraceBlock), 0, s, c->view,
                                 c->q[in].q0, c->q[in].q1, &cnt->qcount[in], &cnt->qcount[out], c->hits,
                                 &cnt->camera_rays, cnt));
        TIMED(K_SHADE, hipLaunchKernelGGL(k_shade, dim3(grid_of(npix, 256)), dim3(256), 0, s, A, c->q[in],
                                          &cnt->qcount[in], c->hits, c->q[out], &cnt->qcount[out], c->V,
                                          &cnt->n_vertices, c->ev0, c->ev1, &cnt->n_events, c->slots,
                                          record ? c->recs : (neb_path_record*)nullptr));
    }
    // deposits
    if (c->prm.density_mode != NEB_DENSITY_ANALYTIC) {
        hipError_t e;
        prof_begin(c, K_OCTREE_INSERT, s);
        if (c->slots)
            e = octree_increment_slots(c->oct, c->V.v0, c->slots, (int32_t)vcap, s);
        else
            e = octree_increment_vertices(c->oct, c->V.v0, &cnt->n_vertices, (int32_t)vcap, s);
        prof_end(c, s);
        HIP_TRY(e);
    }
    // pass 2
    TIMED(K_DENSITY, hipLaunchKernelGGL(k_density, dim3(grid_of(vcap, 256)), dim3(256), 0, s, A, c->V,
                                        &cnt->n_vertices, c->oct.nodes, c->oct.state, c->oct.prm));
    TIMED(K_NEE, hipLaunchKernelGGL(k_nee, dim3(grid_of(vcap, kTraceBlock, 1 << 20)), dim3(kTraceBlock), 0, s, A, c->V,
                                    &cnt->n_vertices,
                                    Images{c->img, c->img + 3 * (size_t)npix, c->img + 6 * (size_t)npix}, c->pq[0],
                                    &cnt->pcount[0], cnt));
    if (A.photons && L >= 3) {
        // merge grid over this iteration's view vertices
        int64_t n = (int64_t)c->G.T * c->G.D + 1;
        prof_begin(c, K_GRID_BUILD, s);
        hipLaunchKernelGGL(k_grid_count, dim3(grid_of(vcap, 256)), dim3(256), 0, s, c->mats, c->V, &cnt->n_vertices, c->G);
        scan_exclusive(c->G.count, c->G.start, n, c->G.sums, s);
        hipLaunchKernelGGL(k_grid_scatter, dim3(grid_of(vcap, 256)), dim3(256), 0, s, c->mats, c->V, &cnt->n_vertices,
                           c->G);
        prof_end(c, s);
        for (int j = 1; j <= L - 2; ++j) {
            int in = (j - 1) & 1, out = j & 1;
            TIMED(K_EXTEND_PHOTON,
                  hipLaunchKernelGGL(k_extend, dim3(grid_of(vcap, kTraceBlock, 1 << 20)), dim3(kTraceBlock), 0, s, c->view,
                                     c->pq[in].p0, c->pq[in].p1, &cnt->pcount[in], &cnt->pcount[out], c->hits,
                                     &cnt->photon_rays, cnt));
            TIMED(K_PHOTON, hipLaunchKernelGGL(k_photon, dim3(grid_of(vcap, 256)), dim3(64), 0, s, A, c->pq[in],
                                               &cnt->pcount[in], c->hits, c->pq[out], &cnt->pcount[out], c->V, c->G,
                                               Images{c->img, c->img + 3 * (size_t)npix, c->img + 6 * (size_t)npix},
                                               cnt));
        }
    }
    // pass 3
    TIMED(K_FINALIZE, hipLaunchKernelGGL(k_finalize, dim3(grid_of(c->ecap, 256)), dim3(256), 0, s, A, c->ev0, c->ev1,
                                         &cnt->n_events, c->V.rho,
                                         Images{c->img, c->img + 3 * (size_t)npix, c->img + 6 * (size_t)npix}));
    hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(1), 0, s, cnt);
    HIP_TRY(hipGetLastError());
    if (record) c->first_iter_recorded = c->iter;
    return NEB_OK;
}

extern "C" neb_status neb_render(neb_ctx c, int32_t n_iterations, void* stream) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (!c->has_scene) return fail(NEB_ERR_STATE, "no scene set");
    if (n_iterations < 0) return fail(NEB_ERR_INVALID_ARG, "negative iteration count");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    for (int i = 0; i < n_iterations; ++i) {
        neb_status st = render_iteration(c, s);
        if (st != NEB_OK) return st;
    }
    return NEB_OK;
}

static neb_status copy_out(neb_ctx c, const float* src_dev, float* dst, int32_t is_dev, float scale, hipStream_t s,
                           int64_t n) {
    if (is_dev) {
        hipLaunchKernelGGL(k_scale_image, dim3(grid_of(n, 256)), dim3(256), 0, s, src_dev, dst, n, scale);
        HIP_TRY(hipGetLastError());
        return NEB_OK;
    }
    std::vector<float> h((size_t)n);
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(h.data(), src_dev, n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) dst[i] = h[i] * scale;
    (void)c;
    return NEB_OK;
}

extern "C" neb_status neb_get_image(neb_ctx c, float* rgb, int32_t is_dev, void* stream) {
    if (!c || !rgb) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    int64_t n = 3 * (int64_t)c->npix;
    float scale = c->iter > 0 ? 1.0f / (float)c->iter : 0.f;
    if (is_dev) {
        hipLaunchKernelGGL(k_mean_image, dim3(grid_of(n, 256)), dim3(256), 0, s, c->img, c->img + n, c->img + 2 * n, rgb,
                           n, scale);
        HIP_TRY(hipGetLastError());
        return NEB_OK;
    }
    std::vector<float> h(3 * (size_t)n);
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(h.data(), c->img, 3 * n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) rgb[i] = (h[i] + h[n + i] + h[2 * n + i]) * scale;
    return NEB_OK;
}

extern "C" neb_status neb_get_technique_images(neb_ctx c, float* e, float* E, float* P, int32_t is_dev, void* stream) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    hipStream_t s = (hipStream_t)stream;
    int64_t n = 3 * (int64_t)c->npix;
    float scale = c->iter > 0 ? 1.0f / (float)c->iter : 0.f;
    float* dst[3] = {e, E, P};
    for (int t = 0; t < 3; ++t)
        if (dst[t]) {
            neb_status st = copy_out(c, c->img + t * n, dst[t], is_dev, scale, s, n);
            if (st != NEB_OK) return st;
        }
    return NEB_OK;
}

extern "C" neb_status neb_query_density(neb_ctx c, const float* pos, const float* nrm, int32_t n, float* out,
                                        int32_t is_dev, void* stream) {
    if (!c || !pos || !nrm || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (n < 0) return fail(NEB_ERR_INVALID_ARG, "negative count");
    if (!c->has_scene) return fail(NEB_ERR_STATE, "no scene set");
    if (n == 0) return NEB_OK;
    hipStream_t s = (hipStream_t)stream;
    if (is_dev) {
        HIP_TRY(octree_density_xyz(c->oct, pos, nrm, n, 1, out, s));
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
        octree_density_xyz(c->oct, dp, dn, n, 1, dout, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(out, dout, 4 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
        st = fail(NEB_ERR_DEVICE, "neb_query_density transfer failed");
    free_list(tmp);
    return st;
}

static neb_status octree_info(const Octree& o, hipStream_t s, int64_t info[8]) {
    OctState st;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(&st, o.state, sizeof(st), hipMemcpyDeviceToHost));
    int32_t used = std::min(st.alloc, o.prm.capacity);
    std::vector<int32_t> nodes((size_t)used);
    HIP_TRY(hipMemcpy(nodes.data(), o.nodes, 4 * (size_t)used, hipMemcpyDeviceToHost));
    int64_t leaf = 0;
    for (int32_t v : nodes)
        if (v >= 0) leaf += v & kOctCountMask;
    info[0] = o.prm.capacity;
    info[1] = used;
    info[2] = st.depth;
    info[3] = leaf - (int64_t)kOctSplitFactor * (int64_t)st.block_iter_sum;
    info[4] = (int64_t)st.deposits;
    info[5] = st.overflow;
    info[6] = st.rejected;
    info[7] = (int64_t)st.lost;
    return NEB_OK;
}

extern "C" neb_status neb_get_stats(neb_ctx c, neb_stats* out) {
    if (!c || !out) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    Counters h;
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    HIP_TRY(hipMemcpy(&h, c->cnt, sizeof(h), hipMemcpyDeviceToHost));
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
    out->bvh_nodes = (int64_t)h.bvh_nodes;
    out->bvh_tris = (int64_t)h.bvh_tris;
    out->photon_items = (int64_t)h.photon_items;
    out->photon_continued = (int64_t)h.photon_continued;
    out->grid_cells = (int64_t)h.grid_cells;
    out->candidates = (int64_t)h.candidates;
    if (c->has_scene) {
        int64_t info[8];
        neb_status st = octree_info(c->oct, c->last_stream, info);
        if (st != NEB_OK) return st;
        out->oct_capacity = info[0];
        out->oct_allocated = info[1];
        out->oct_depth = info[2];
        out->oct_ledger = info[3];
        out->oct_deposits = info[4];
        out->oct_overflow = info[5];
        out->oct_rejected = info[6];
        out->oct_lost = info[7];
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

extern "C" neb_status neb_get_octree(neb_ctx c, int32_t* nodes, int32_t cap, int64_t info[8]) {
    if (!c || !info) return fail(NEB_ERR_INVALID_ARG, "null pointer");
    if (!c->has_scene) return fail(NEB_ERR_STATE, "no scene set");
    neb_status st = octree_info(c->oct, c->last_stream, info);
    if (st != NEB_OK) return st;
    if (nodes && cap > 0)
        HIP_TRY(hipMemcpy(nodes, c->oct.nodes, 4 * (size_t)std::min(cap, c->oct.prm.capacity), hipMemcpyDeviceToHost));
    return NEB_OK;
}

extern "C" neb_status neb_profile_kernels(neb_ctx c, int32_t enable) {
    if (!c) return fail(NEB_ERR_INVALID_ARG, "null context");
    if (enable) {
        if (c->prof_ev.empty()) {
            c->prof_ev.resize(4096);
            c->prof_kid.resize(2048);
            for (auto& e : c->prof_ev) HIP_TRY(hipEventCreate(&e));
        }
        prof_harvest(c);
        for (int k = 0; k < 32; ++k) {
            c->prof_ms[k] = 0.0;
            c->prof_launches[k] = 0;
        }
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
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(9 * (int64_t)c->npix, 256)), dim3(256), 0, nullptr, c->img, 0.f,
                       9 * (int64_t)c->npix);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, nullptr, (int32_t*)c->cnt, 0, (int64_t)(sizeof(Counters) / 4));
    if (c->has_scene) HIP_TRY(octree_init_nodes(c->oct, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    c->iter = 0;
    c->first_iter_recorded = 0;
    return NEB_OK;
}

extern "C" void neb_destroy(neb_ctx c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    free_list(c->scene_allocs);
    free_list(c->allocs);
    c->oct.nodes = nullptr;   // owned by allocs
    c->oct.state = nullptr;
    octree_release(c->oct);
    for (auto& e : c->prof_ev) (void)hipEventDestroy(e);
    delete c;
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
    octree_params_init(o->o.prm, scene_min, scene_max, capacity);
    o->o.last_iter = 1;
    hipError_t e = hipMalloc(&o->o.nodes, 4 * (size_t)o->o.prm.capacity);
    if (e == hipSuccess) e = hipMalloc(&o->o.state, sizeof(OctState));
    if (e == hipSuccess) e = octree_init_nodes(o->o, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        octree_release(o->o);
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
    octree_params_set_iteration(o->o.prm, iter);
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
    neb_status st = octree_info(o->o, (hipStream_t)stream, info);
    if (st != NEB_OK) return st;
    if (nodes && cap > 0)
        HIP_TRY(hipMemcpy(nodes, o->o.nodes, 4 * (size_t)std::min(cap, o->o.prm.capacity), hipMemcpyDeviceToHost));
    return NEB_OK;
}

extern "C" void neb_octree_destroy(neb_octree o) {
    if (!o) return;
    (void)hipDeviceSynchronize();
    octree_release(o->o);
    delete o;
}
