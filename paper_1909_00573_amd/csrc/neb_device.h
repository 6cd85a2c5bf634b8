// Device helpers of libneb: vector math, Philox, BSDFs, plane-box area,
// octree addressing and queries, BVH traversal.  gfx950 only.
#pragma once
#include "neb_internal.h"

namespace neb {

#define NEB_PI 3.14159265358979323846f

struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mk3(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ f3 operator-(f3 a) { return mk3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return mk3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ f3 operator*(f3 a, f3 b) { return mk3(a.x * b.x, a.y * b.y, a.z * b.z); }
__device__ __forceinline__ float dot3(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross3(f3 a, f3 b) {
    return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ f3 normalize3(f3 a) { return a * rsqrtf(dot3(a, a)); }
__device__ __forceinline__ f3 xyz(float4 v) { return mk3(v.x, v.y, v.z); }
__device__ __forceinline__ float4 f4(f3 a, float w) { return make_float4(a.x, a.y, a.z, w); }
__device__ __forceinline__ float get3(f3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
__device__ __forceinline__ bool is_zero3(f3 a) { return a.x == 0.f && a.y == 0.f && a.z == 0.f; }
__device__ __forceinline__ f3 load3(const float* p) { return mk3(p[0], p[1], p[2]); }

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t hi0 = __umulhi(m0, c.x), lo0 = m0 * c.x;
        uint32_t hi1 = __umulhi(m1, c.z), lo1 = m1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

struct U4 {
    float u[4];
};
// four uniforms in [0,1): the top 24 bits of each output, exact in FP32
__device__ __forceinline__ U4 uniforms(uint32_t k0, uint32_t k1, uint32_t a, uint32_t b, uint32_t c,
                                       uint32_t tag) {
    uint4 x = philox10(make_uint4(a, b, c, tag), k0, k1);
    const float s = 1.0f / 16777216.0f;
    U4 r;
    r.u[0] = (float)(x.x >> 8) * s;
    r.u[1] = (float)(x.y >> 8) * s;
    r.u[2] = (float)(x.z >> 8) * s;
    r.u[3] = (float)(x.w >> 8) * s;
    return r;
}

// branchless orthonormal basis around n (Duff et al., JCGT 6(1), 2017)
__device__ __forceinline__ void basis(f3 n, f3& t1, f3& t2) {
    float sg = copysignf(1.0f, n.z);
    float a = -1.0f / (sg + n.z);
    float b = n.x * n.y * a;
    t1 = mk3(1.0f + sg * n.x * n.x * a, sg * b, -sg * n.x);
    t2 = mk3(b, sg + n.y * n.y * a, -n.y);
}

// ---------------------------------------------------------------------------
// BSDFs.  Geometric normal only; wi = direction the path arrived from, wo =
// direction it leaves to, both pointing away from the surface.  Delta lobes
// report their discrete selection probability as pdf.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool mat_delta(int type) { return type == NEB_MAT_MIRROR || type == NEB_MAT_DIELECTRIC; }
__device__ __forceinline__ bool mat_black(const neb_material& m) {
    return m.albedo[0] == 0.f && m.albedo[1] == 0.f && m.albedo[2] == 0.f;
}
__device__ __forceinline__ bool mat_emits(const neb_material& m) {
    return m.emission[0] + m.emission[1] + m.emission[2] > 0.f;
}

__device__ __forceinline__ float fresnel(float cos_i, float eta) {
    float s2 = eta * eta * (1.0f - cos_i * cos_i);
    if (s2 >= 1.0f) return 1.0f;
    float ct = sqrtf(1.0f - s2);
    float rs = (eta * cos_i - ct) / (eta * cos_i + ct);
    float rp = (cos_i - eta * ct) / (cos_i + eta * ct);
    return 0.5f * (rs * rs + rp * rp);
}

__device__ __forceinline__ float ggx_d(float a, float c) {
    if (c <= 0.f) return 0.f;
    float a2 = a * a;
    float t = c * c * (a2 - 1.0f) + 1.0f;
    return a2 / (NEB_PI * t * t);
}
__device__ __forceinline__ float ggx_g1(float a, float c) {
    float c2 = c * c;
    return 2.0f / (1.0f + sqrtf(1.0f + a * a * (1.0f - c2) / c2));
}

__device__ __forceinline__ float bsdf_pdf(const neb_material& m, f3 n, f3 wi, f3 wo) {
    float ci = dot3(n, wi), co = dot3(n, wo);
    bool same = ci * co > 0.f;
    switch (m.type) {
    case NEB_MAT_LAMBERT: return same ? fabsf(co) * (1.0f / NEB_PI) : 0.f;
    case NEB_MAT_MIRROR: return same ? 1.f : 0.f;
    case NEB_MAT_DIELECTRIC: {
        float F = fresnel(fabsf(ci), ci > 0.f ? 1.0f / m.ior : m.ior);
        return same ? F : 1.0f - F;
    }
    case NEB_MAT_GGX: {
        if (!same) return 0.f;
        f3 ns = ci > 0.f ? n : -n;
        f3 h = normalize3(wi + wo);
        float cm = dot3(h, ns);
        return ggx_d(m.alpha, cm) * cm / (4.0f * fabsf(dot3(wo, h)));
    }
    }
    return 0.f;
}

__device__ __forceinline__ f3 bsdf_f(const neb_material& m, f3 n, f3 wi, f3 wo) {
    float ci = dot3(n, wi), co = dot3(n, wo);
    f3 alb = load3(m.albedo);
    if (ci * co <= 0.f) return mk3(0.f, 0.f, 0.f);
    if (m.type == NEB_MAT_LAMBERT) return alb * (1.0f / NEB_PI);
    if (m.type == NEB_MAT_GGX) {
        f3 ns = ci > 0.f ? n : -n;
        f3 h = normalize3(wi + wo);
        float D = ggx_d(m.alpha, dot3(h, ns));
        float G = ggx_g1(m.alpha, fabsf(ci)) * ggx_g1(m.alpha, fabsf(co));
        return alb * (D * G / (4.0f * fabsf(ci) * fabsf(co)));
    }
    return mk3(0.f, 0.f, 0.f);
}

struct Sample {
    f3 dir, w;
    float pdf;
    int ev;      // 1 scatter, 2 reflect, 3 refract, 0 failed
};

__device__ __forceinline__ Sample bsdf_sample(const neb_material& m, f3 n, f3 wi, const U4& u) {
    Sample s;
    s.ev = 0;
    s.pdf = 0.f;
    s.w = mk3(0.f, 0.f, 0.f);
    s.dir = mk3(0.f, 0.f, 1.f);
    float ci = dot3(n, wi);
    if (ci == 0.f) return s;
    f3 ns = ci > 0.f ? n : -n;
    f3 alb = load3(m.albedo);
    if (m.type == NEB_MAT_LAMBERT) {
        f3 t1, t2;
        basis(ns, t1, t2);
        float r = sqrtf(u.u[1]);
        float sp, cp;
        sincosf(2.0f * NEB_PI * u.u[2], &sp, &cp);
        float z = sqrtf(fmaxf(0.f, 1.0f - u.u[1]));
        s.dir = normalize3(t1 * (r * cp) + t2 * (r * sp) + ns * z);
        float co = dot3(s.dir, ns);
        if (co <= 0.f) return s;
        s.pdf = co * (1.0f / NEB_PI);
        s.w = alb;
        s.ev = 1;
    } else if (m.type == NEB_MAT_MIRROR) {
        float c = dot3(wi, ns);
        s.dir = ns * (2.0f * c) - wi;
        s.pdf = 1.0f;
        s.w = alb;
        s.ev = 2;
    } else if (m.type == NEB_MAT_DIELECTRIC) {
        float c = dot3(wi, ns);
        float eta = ci > 0.f ? 1.0f / m.ior : m.ior;
        float F = fresnel(c, eta);
        if (u.u[0] < F) {
            s.dir = ns * (2.0f * c) - wi;
            s.pdf = F;
            s.ev = 2;
        } else {
            float ct = sqrtf(fmaxf(0.f, 1.0f - eta * eta * (1.0f - c * c)));
            s.dir = normalize3(ns * (eta * c - ct) - wi * eta);
            s.pdf = 1.0f - F;
            s.ev = 3;
        }
        s.w = alb;
    } else if (m.type == NEB_MAT_GGX) {
        float a = m.alpha;
        float tt = a * sqrtf(u.u[1] / (1.0f - u.u[1]));
        float ct = rsqrtf(1.0f + tt * tt);
        float st = tt * ct;
        float sp, cp;
        sincosf(2.0f * NEB_PI * u.u[2], &sp, &cp);
        f3 t1, t2;
        basis(ns, t1, t2);
        f3 h = normalize3(t1 * (st * cp) + t2 * (st * sp) + ns * ct);
        float wh = dot3(wi, h);
        if (wh <= 0.f) return s;
        s.dir = h * (2.0f * wh) - wi;
        float co = dot3(s.dir, ns);
        if (co <= 0.f) return s;
        float cim = fabsf(ci);
        float G = ggx_g1(a, cim) * ggx_g1(a, co);
        s.pdf = ggx_d(a, ct) * ct / (4.0f * wh);
        s.w = alb * (G * wh / (cim * ct));
        s.ev = 1;
    }
    return s;
}

// ---------------------------------------------------------------------------
// eq. (area): area of the plane (p, n) inside the box [bmin, bmax].  The plane
// offset is taken relative to the box's min corner; the 3-D case sums in FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float plane_box_area(f3 bmin, f3 bmax, f3 p, f3 n) {
    f3 s = bmax - bmin;
    f3 a = mk3(fabsf(n.x), fabsf(n.y), fabsf(n.z));
    if (fabsf(a.x - 1.0f) < 1e-3f) return s.y * s.z;
    if (fabsf(a.y - 1.0f) < 1e-3f) return s.x * s.z;
    if (fabsf(a.z - 1.0f) < 1e-3f) return s.x * s.y;
    f3 q = p - bmin;
    for (int d = 0; d < 3; ++d) {
        if (get3(a, d) < 1e-4f) {
            int ix = d == 0 ? 1 : (d == 1 ? 2 : 0);
            int iy = d == 0 ? 2 : (d == 1 ? 0 : 1);
            float nx = get3(n, ix), ny = get3(n, iy);
            float ex = nx * get3(s, ix), ey = ny * get3(s, iy);
            float t = nx * get3(q, ix) + ny * get3(q, iy);
            float sum = fmaxf(0.f, t) - fmaxf(0.f, t - ex) - fmaxf(0.f, t - ey) + fmaxf(0.f, t - ex - ey);
            return get3(s, d) * fabsf(sum / (nx * ny));
        }
    }
    double ex = (double)n.x * s.x, ey = (double)n.y * s.y, ez = (double)n.z * s.z;
    double t = (double)n.x * q.x + (double)n.y * q.y + (double)n.z * q.z;
    double sum = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        double h = t - ((c & 1) ? ex : 0.0) - ((c & 2) ? ey : 0.0) - ((c & 4) ? ez : 0.0);
        double v = h > 0.0 ? h * h : 0.0;
        sum += (__popc(c) & 1) ? -v : v;
    }
    return (float)fabs(sum / (2.0 * (double)n.x * (double)n.y * (double)n.z));
}

// ---------------------------------------------------------------------------
// Octree addressing (FP32, no contraction, as the class of Appendix B) and
// the density query of eq. (octdensity).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool oct_norm(const OctParams& P, f3 p, float q[3]) {
    float pv[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float v = __fmul_rn(__fsub_rn(pv[i], P.min_bound[i]), P.size_inv[i]);
        if (!(v >= 0.0f && v < 1.0f)) return false;
        q[i] = v;
    }
    return true;
}

// A point's cell at the octree's finest level: integer coordinates
// floor(q * 2^depth) of its normalised position q.  The leaf reached at level
// L holds the cell c >> (depth - L); the child taken below level L is bit
// depth - L - 1 of each coordinate (the same child as the deposits take from
// floor(q * 2^(L+1)) & 1, as scaling by a power of two is exact).
struct OctCell {
    int32_t c[3];
};

__device__ __forceinline__ bool oct_cell(const OctParams& P, int depth, f3 p, OctCell& k) {
    float q[3];
    if (!oct_norm(P, p, q)) return false;
    const float fine = (float)(1 << depth);
#pragma unroll
    for (int a = 0; a < 3; ++a) k.c[a] = (int32_t)(q[a] * fine);
    return true;
}

// the node word below inner node word w (< 0) on the way to cell k, `shift`
// = depth - (level of the child)
__device__ __forceinline__ int32_t oct_child(const int32_t* __restrict__ nodes, int32_t w, const OctCell& k,
                                             int shift) {
    const int32_t child = ((k.c[0] >> shift) & 1) | (((k.c[1] >> shift) & 1) << 1) | (((k.c[2] >> shift) & 1) << 2);
    return nodes[child - w];
}

// Floor under the area of the surface inside a leaf of diagonal `diag`, so
// that a surface grazing a cell does not give an unbounded density: a tenth
// of diag^2 for the probe at the query point, a hundredth for the offset
// probes (Appendix B).
__device__ __forceinline__ float oct_area_floor(float diag, bool centre) {
    return diag * diag * (centre ? 0.1f : 0.01f);
}

// eq. (octdensity) at the leaf (word w, level `level`) holding cell k of the
// point p with normal n: the leaf's count over the area of the plane through
// p inside the leaf's box (eq. area), times the density scale.  centre: the
// probe at the query point; then *diag_out receives the leaf's diagonal (if
// the leaf has a count).
__device__ __forceinline__ float oct_leaf_density(const OctParams& P, float density_scale, int depth,
                                                  const OctCell& k, int level, int32_t w, f3 p, f3 n, bool centre,
                                                  float* diag_out) {
    const int32_t count = w & kOctCountMask;
    if (count <= 0) return 0.f;
    const int32_t cells = 1 << level;  // per axis at this level
    const int shift = depth - level;
    float edge[3], lo[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        edge[a] = 1.0f / ((float)cells * P.size_inv[a]);
        lo[a] = (float)(k.c[a] >> shift) * edge[a];
    }
    const f3 bmin = mk3(lo[0], lo[1], lo[2]);
    const f3 bmax = bmin + mk3(edge[0], edge[1], edge[2]);
    const f3 rel = mk3(p.x - P.min_bound[0], p.y - P.min_bound[1], p.z - P.min_bound[2]);
    const float area = plane_box_area(bmin, bmax, rel, n);
    const float diag = P.scene_scale / (float)cells;
    if (centre) *diag_out = diag;
    return density_scale * (float)count / fmaxf(oct_area_floor(diag, centre), area);
}

// upper median of n (1..5) values: the (n/2)-th smallest (sorts v)
__device__ __forceinline__ float upper_median(float* v, int n) {
    for (int i = 1; i < n; ++i) {
        const float x = v[i];
        int j = i;
        for (; j > 0 && v[j - 1] > x; --j) v[j] = v[j - 1];
        v[j] = x;
    }
    return v[n / 2];
}

// eq. (octdensity) at the leaf holding p (Appendix B get_density)
__device__ __forceinline__ float oct_query(const int32_t* __restrict__ nodes, const OctParams& P, float density_scale,
                                           int depth, f3 p, f3 n, bool centre, float* diag_out) {
    OctCell k;
    if (!oct_cell(P, depth, p, k)) return 0.f;
    int32_t w = nodes[P.root];
    int level = 0;
    while (w < 0) {
        ++level;
        w = oct_child(nodes, w, k, depth - level);
    }
    return oct_leaf_density(P, density_scale, depth, k, level, w, p, n, centre, diag_out);
}

// Appendix B get_density_robust: the densities at p and at four points
// offset along the tangents by 1.1 leaf diagonals of p's leaf (1.1e-3
// scene units when that leaf is empty); the upper median of the non-zero
// ones (0 if none)
__device__ __forceinline__ float oct_query_robust(const int32_t* __restrict__ nodes, const OctParams& P,
                                                  float density_scale, int depth, f3 p, f3 n) {
    f3 tx, ty;
    basis(n, tx, ty);
    float diag = 1e-3f;
    float found[5];
    int nf = 0;
    const float centre = oct_query(nodes, P, density_scale, depth, p, n, true, &diag);
    if (centre > 0.f) found[nf++] = centre;
    const float step = diag * 1.1f;
    const f3 probe[4] = {p + tx * step, p - tx * step, p + ty * step, p - ty * step};
    // the four offset probes descend together, one level per step, so that
    // their node loads are in flight at once (a probe outside the octree's
    // box stops at once with density 0)
    OctCell k[4];
    int32_t w[4];
    int level[4];
    const int32_t root = nodes[P.root];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool in = oct_cell(P, depth, probe[i], k[i]);
        if (!in) k[i].c[0] = k[i].c[1] = k[i].c[2] = 0;
        w[i] = in ? root : 0;
        level[i] = 0;
    }
    while (w[0] < 0 || w[1] < 0 || w[2] < 0 || w[3] < 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (w[i] < 0) {
                ++level[i];
                w[i] = oct_child(nodes, w[i], k[i], depth - level[i]);
            }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float r = oct_leaf_density(P, density_scale, depth, k[i], level[i], w[i], probe[i], n, false, nullptr);
        if (r > 0.f) found[nf++] = r;
    }
    return nf ? upper_median(found, nf) : 0.f;
}

// ---------------------------------------------------------------------------
// BVH traversal: four child boxes per 128-byte node, per-lane stack in LDS,
// watertight ray-triangle test (Woop, Benthin, Wald, JCGT 2(1), 2013).
// ---------------------------------------------------------------------------
struct RayPre {
    f3 o, d, inv;
    int kx, ky, kz;
    float sx, sy, sz;
};

__device__ __forceinline__ RayPre ray_pre(f3 o, f3 d) {
    RayPre r;
    r.o = o;
    r.d = d;
    const float big = 1e30f;
    r.inv = mk3(fabsf(d.x) > 1e-30f ? 1.0f / d.x : copysignf(big, d.x),
                fabsf(d.y) > 1e-30f ? 1.0f / d.y : copysignf(big, d.y),
                fabsf(d.z) > 1e-30f ? 1.0f / d.z : copysignf(big, d.z));
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    if (get3(d, kz) < 0.f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    float dz = get3(d, kz);
    r.sx = get3(d, kx) / dz;
    r.sy = get3(d, ky) / dz;
    r.sz = 1.0f / dz;
    return r;
}

// returns t in (0, tmax) or -1
__device__ __forceinline__ float tri_hit(const RayPre& r, f3 v0, f3 v1, f3 v2, float tmax) {
    f3 A = v0 - r.o, B = v1 - r.o, C = v2 - r.o;
    float az = get3(A, r.kz), bz = get3(B, r.kz), cz = get3(C, r.kz);
    float Ax = get3(A, r.kx) - r.sx * az, Ay = get3(A, r.ky) - r.sy * az;
    float Bx = get3(B, r.kx) - r.sx * bz, By = get3(B, r.ky) - r.sy * bz;
    float Cx = get3(C, r.kx) - r.sx * cz, Cy = get3(C, r.ky) - r.sy * cz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.f || V == 0.f || W == 0.f) {
        U = (float)((double)Cx * By - (double)Cy * Bx);
        V = (float)((double)Ax * Cy - (double)Ay * Cx);
        W = (float)((double)Bx * Ay - (double)By * Ax);
    }
    if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return -1.f;
    float det = U + V + W;
    if (det == 0.f) return -1.f;
    float T = U * (r.sz * az) + V * (r.sz * bz) + W * (r.sz * cz);
    float t = T / det;
    return (t > 0.f && t < tmax) ? t : -1.f;
}

__device__ __forceinline__ bool box_hit(const RayPre& r, float lx, float ly, float lz, float hx, float hy,
                                        float hz, float tmax, float& tn) {
    float t0x = (lx - r.o.x) * r.inv.x, t1x = (hx - r.o.x) * r.inv.x;
    float t0y = (ly - r.o.y) * r.inv.y, t1y = (hy - r.o.y) * r.inv.y;
    float t0z = (lz - r.o.z) * r.inv.z, t1z = (hz - r.o.z) * r.inv.z;
    float tnear = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    float tfar = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    tn = tnear;
    return tnear <= tfar * 1.00000024f;
}

// Resumable closest-hit traversal: the state of one ray, advanced by up to
// max_steps node visits per call, so a lane whose ray ends can take a new
// one while the rest of its wave is still traversing.  Ties on t go to the
// lowest primitive id; the stack is the lane's kStack LDS slots, stride
// kTraceBlock (the BVH's stack need must be below kStack); kAnyHit stops at
// the first hit below tmax.
struct TraceState {
    RayPre r;
    float best;
    int prim;
    int node;
    int sp;
};

__device__ __forceinline__ void trace_begin(TraceState& T, int root, f3 o, f3 d, float tmax = INFINITY) {
    T.r = ray_pre(o, d);
    T.best = tmax;
    T.prim = -1;
    T.node = root;
    T.sp = 0;
}

// returns true when the ray is done (T.best, T.prim hold the closest hit
// below the tmax of trace_begin; kAnyHit: T.prim >= 0 once any hit below
// tmax is found, which ends the ray)
// (distance, node) pair of a child still to visit; compare-exchange by distance
__device__ __forceinline__ void near_first(float& da, int& na, float& db, int& nb) {
    const bool sw = db < da;
    const float d = sw ? db : da;
    const int n = sw ? nb : na;
    db = sw ? da : db;
    nb = sw ? na : nb;
    da = d;
    na = n;
}

template <int kStack, bool kAnyHit = false>
__device__ __forceinline__ bool trace_steps(const SceneView& S, TraceState& T, int* stack, int max_steps,
                                            unsigned& nodes, unsigned& tris) {
    const RayPre& r = T.r;
    for (int step = 0; step < max_steps; ++step) {
        // one 128-byte node: the four children's boxes coordinate by
        // coordinate, their links and leaf counts
        const float4* nd = S.bvh + 8 * T.node;
        ++nodes;
        const float4 lx = nd[0], ly = nd[1], lz = nd[2], hx = nd[3], hy = nd[4], hz = nd[5];
        const int4 lk = *reinterpret_cast<const int4*>(nd + 6);
        const int4 ct = *reinterpret_cast<const int4*>(nd + 7);
        float t0, t1, t2, t3;
        const bool h0 = box_hit(r, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, T.best, t0) && lk.x >= 0;
        const bool h1 = box_hit(r, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, T.best, t1) && lk.y >= 0;
        const bool h2 = box_hit(r, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, T.best, t2) && lk.z >= 0;
        const bool h3 = box_hit(r, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, T.best, t3) && lk.w >= 0;
        // the hit leaf children's triangles in one loop, each triangle's
        // three words loaded one iteration ahead of its test, so that the
        // leaves of a node cost one load latency, not one per triangle
        const int n0 = (h0 && ct.x > 0) ? ct.x : 0, n1 = (h1 && ct.y > 0) ? ct.y : 0;
        const int n2 = (h2 && ct.z > 0) ? ct.z : 0, n3 = (h3 && ct.w > 0) ? ct.w : 0;
        const int e0 = n0, e1 = e0 + n1, e2 = e1 + n2, nt = e2 + n3;
        if (nt > 0) {
            tris += nt;
            // m-th triangle of the hit leaves, slot by slot
            auto tri_of = [&](int m) {
                return m < e0 ? lk.x + m : (m < e1 ? lk.y + (m - e0) : (m < e2 ? lk.z + (m - e1) : lk.w + (m - e2)));
            };
            const float4* tp = S.tri + 3 * tri_of(0);
            float4 p0 = tp[0], p1 = tp[1], p2 = tp[2];
            for (int m = 0; m < nt; ++m) {
                float4 q0 = p0, q1 = p1, q2 = p2;
                if (m + 1 < nt) {
                    const float4* tq = S.tri + 3 * tri_of(m + 1);
                    q0 = tq[0];
                    q1 = tq[1];
                    q2 = tq[2];
                }
                float t = tri_hit(r, xyz(p0), xyz(p1), xyz(p2), kAnyHit ? T.best : T.best * 1.0000001f);
                int id = __float_as_int(p0.w);
                if (t > 0.f && (t < T.best || (t == T.best && id < T.prim))) {
                    T.best = t;
                    T.prim = id;
                    if (kAnyHit) return true;
                }
                p0 = q0;
                p1 = q1;
                p2 = q2;
            }
        }
        // inner children still in reach, sorted nearest first (five
        // compare-exchanges); the nearest is next, the others are pushed
        // farthest first
        float d0 = (h0 && ct.x == 0 && t0 < T.best) ? t0 : INFINITY;
        float d1 = (h1 && ct.y == 0 && t1 < T.best) ? t1 : INFINITY;
        float d2 = (h2 && ct.z == 0 && t2 < T.best) ? t2 : INFINITY;
        float d3 = (h3 && ct.w == 0 && t3 < T.best) ? t3 : INFINITY;
        const int k = (d0 < INFINITY) + (d1 < INFINITY) + (d2 < INFINITY) + (d3 < INFINITY);
        if (k == 0) {
            if (T.sp == 0) return true;
            T.node = stack[(--T.sp) * kTraceBlock];
            continue;
        }
        int c0 = lk.x, c1 = lk.y, c2 = lk.z, c3 = lk.w;
        near_first(d0, c0, d1, c1);
        near_first(d2, c2, d3, c3);
        near_first(d0, c0, d2, c2);
        near_first(d1, c1, d3, c3);
        near_first(d1, c1, d2, c2);
        if (k > 3 && T.sp < kStack) stack[(T.sp++) * kTraceBlock] = c3;
        if (k > 2 && T.sp < kStack) stack[(T.sp++) * kTraceBlock] = c2;
        if (k > 1 && T.sp < kStack) stack[(T.sp++) * kTraceBlock] = c1;
        T.node = c0;
    }
    return false;
}

// device-wide counter add with one atomic per wave
__device__ __forceinline__ void wave_add_u64(unsigned long long* dst, unsigned v) {
    unsigned long long s = v;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(dst, s);
}

// this block's stripe of the work statistics
__device__ __forceinline__ StatLine& stat_line(Counters* c) { return c->st[blockIdx.x & (kStatStripes - 1)]; }

// Block-wide slot reservation in one queue whose tail is *counter: one
// atomic per block (the waves' counts meet in wc[kWaves] and bb, LDS).  Every
// thread of the block must call it; lanes with take == false get -1.
template <int kWaves>
__device__ __forceinline__ int block_reserve(int32_t* counter, bool take, int* wc, int* bb) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long m = __ballot(take);
    if (lane == 0) wc[wid] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += wc[w];
        *bb = tot ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    int base = *bb;
    for (int w = 0; w < wid; ++w) base += wc[w];
    __syncthreads();  // wc and bb are rewritten by the next call
    return take ? base + __popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// wave-aggregated slot reservation: returns this lane's index in a queue
// whose tail is *counter; lanes with take == false get -1
__device__ __forceinline__ int wave_reserve(int* counter, bool take) {
    unsigned long long mask = __ballot(take);
    int lane = threadIdx.x & 63;
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (mask == 0) return -1;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader, 64);
    unsigned long long below = mask & ((1ull << lane) - 1ull);
    return take ? base + __popcll(below) : -1;
}

}  // namespace neb
