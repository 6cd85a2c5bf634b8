// Host check of the BVH builder's four-wide nodes (test infrastructure).
// Reads a mesh (int32 nv, nt; nv*3 float32 vertices; nt*3 int32 indices),
// builds the tree and prints one line of key=value figures:
//   nodes, stack_need, box_violations (a triangle vertex or a grandchild box
//   outside the box its parent stores for it), unseen (triangles not placed
//   exactly once), orphans (nodes without exactly one parent), rays, hits,
//   differing (closest hit of the tree walk != brute force over every
//   triangle, both with the same watertight test), max_stack (deepest stack
//   the walk reached; must not exceed stack_need).
#include "neb_bvh.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <utility>
#include <vector>

using neb::BvhHost;

namespace {

struct V3 {
    float x, y, z;
};
float at(const V3& v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// watertight ray-triangle test (Woop, Benthin, Wald, JCGT 2(1), 2013)
struct Ray {
    V3 o, inv;
    int kx, ky, kz;
    float sx, sy, sz;
};
Ray make_ray(V3 o, V3 d) {
    Ray r;
    r.o = o;
    auto rcp = [](float x) { return fabsf(x) > 1e-30f ? 1.f / x : copysignf(1e30f, x); };
    r.inv = {rcp(d.x), rcp(d.y), rcp(d.z)};
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    r.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    r.kx = (r.kz + 1) % 3;
    r.ky = (r.kx + 1) % 3;
    if (at(d, r.kz) < 0.f) std::swap(r.kx, r.ky);
    r.sx = at(d, r.kx) / at(d, r.kz);
    r.sy = at(d, r.ky) / at(d, r.kz);
    r.sz = 1.f / at(d, r.kz);
    return r;
}
float hit_tri(const Ray& r, const float* t, float tmax) {
    V3 a{t[0] - r.o.x, t[1] - r.o.y, t[2] - r.o.z}, b{t[4] - r.o.x, t[5] - r.o.y, t[6] - r.o.z},
        c{t[8] - r.o.x, t[9] - r.o.y, t[10] - r.o.z};
    float az = at(a, r.kz), bz = at(b, r.kz), cz = at(c, r.kz);
    float ax = at(a, r.kx) - r.sx * az, ay = at(a, r.ky) - r.sy * az;
    float bx = at(b, r.kx) - r.sx * bz, by = at(b, r.ky) - r.sy * bz;
    float cx = at(c, r.kx) - r.sx * cz, cy = at(c, r.ky) - r.sy * cz;
    double u = (double)cx * by - (double)cy * bx, v = (double)ax * cy - (double)ay * cx,
           w = (double)bx * ay - (double)by * ax;
    if ((u < 0 || v < 0 || w < 0) && (u > 0 || v > 0 || w > 0)) return -1.f;
    double det = u + v + w;
    if (det == 0) return -1.f;
    float tt = (float)((u * az + v * bz + w * cz) * r.sz / det);
    return (tt > 0.f && tt < tmax) ? tt : -1.f;
}
// slab test with a small outward tolerance; tn = entry distance
bool hit_box(const Ray& r, const float* lo, const float* hi, float tmax, float& tn) {
    float t0 = 0.f, t1 = tmax;
    const float o[3] = {r.o.x, r.o.y, r.o.z}, iv[3] = {r.inv.x, r.inv.y, r.inv.z};
    for (int a = 0; a < 3; ++a) {
        float u = (lo[a] - o[a]) * iv[a], v = (hi[a] - o[a]) * iv[a];
        t0 = std::max(t0, std::min(u, v));
        t1 = std::min(t1, std::max(u, v));
    }
    tn = t0;
    return t0 <= t1 * 1.0000003f;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t n[2];
    if (fread(n, 4, 2, f) != 2) return 2;
    std::vector<float> vert(3 * (size_t)n[0]);
    std::vector<int32_t> idx(3 * (size_t)n[1]);
    if (fread(vert.data(), 4, vert.size(), f) != vert.size() || fread(idx.data(), 4, idx.size(), f) != idx.size())
        return 2;
    fclose(f);
    BvhHost H;
    if (!neb::build_bvh(vert.data(), n[0], idx.data(), n[1], H)) return 3;
    auto node = [&](int i) { return &H.nodes[32 * (size_t)i]; };
    auto links = [&](int i, int32_t* lk, int32_t* ct) {
        std::memcpy(lk, node(i) + 24, 16);
        std::memcpy(ct, node(i) + 28, 16);
    };
    long bad = 0;
    std::vector<int> seen(n[1], 0), parents(H.n_nodes, 0);
    for (int i = 0; i < H.n_nodes; ++i) {
        int32_t lk[4], ct[4];
        links(i, lk, ct);
        for (int c = 0; c < 4; ++c) {
            if (lk[c] < 0) continue;
            const float* d = node(i);
            const float lo[3] = {d[c], d[4 + c], d[8 + c]}, hi[3] = {d[12 + c], d[16 + c], d[20 + c]};
            if (ct[c] > 0) {
                for (int m = 0; m < ct[c]; ++m) {
                    const float* t = &H.tris[12 * (size_t)(lk[c] + m)];
                    int32_t pid;
                    std::memcpy(&pid, t + 3, 4);
                    if (pid >= 0 && pid < n[1]) seen[pid]++;
                    for (int k = 0; k < 3; ++k)
                        for (int a = 0; a < 3; ++a) bad += t[4 * k + a] < lo[a] || t[4 * k + a] > hi[a];
                }
            } else {
                parents[lk[c]]++;
                int32_t lk2[4], ct2[4];
                links(lk[c], lk2, ct2);
                const float* e = node(lk[c]);
                for (int c2 = 0; c2 < 4; ++c2)
                    if (lk2[c2] >= 0)
                        for (int a = 0; a < 3; ++a) bad += e[4 * a + c2] < lo[a] || e[12 + 4 * a + c2] > hi[a];
            }
        }
    }
    long unseen = 0, orphans = 0;
    for (int p = 0; p < n[1]; ++p) unseen += seen[p] != 1;
    for (int i = 1; i < H.n_nodes; ++i) orphans += parents[i] != 1;

    float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
    for (int i = 0; i < n[0]; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], vert[3 * i + a]);
            hi[a] = std::max(hi[a], vert[3 * i + a]);
        }
    std::mt19937 rng(5);
    std::uniform_real_distribution<float> U(0.f, 1.f);
    const int nr = atoi(argv[2]);
    long hits = 0, differing = 0;
    int max_stack = 0;
    for (int q = 0; q < nr; ++q) {
        V3 o{lo[0] + U(rng) * (hi[0] - lo[0]), lo[1] + U(rng) * (hi[1] - lo[1]), lo[2] + U(rng) * (hi[2] - lo[2])};
        float z = 2.f * U(rng) - 1.f, ph = 6.2831853f * U(rng), s = sqrtf(std::max(0.f, 1.f - z * z));
        Ray r = make_ray(o, {s * cosf(ph), s * sinf(ph), z});
        auto better = [](float t, int id, float bt, int bp) { return t > 0.f && (t < bt || (t == bt && id < bp)); };
        float bt = INFINITY;
        int bp = -1;
        for (int p = 0; p < n[1]; ++p) {
            const float* t = &H.tris[12 * (size_t)p];
            int32_t id;
            std::memcpy(&id, t + 3, 4);
            float tt = hit_tri(r, t, bt * 1.0000001f);
            if (better(tt, id, bt, bp)) bt = tt, bp = id;
        }
        // the tree walk: nearest inner child next, the others pushed
        float best = INFINITY;
        int prim = -1, nd = 0;
        std::vector<int> stack;
        for (;;) {
            int32_t lk[4], ct[4];
            links(nd, lk, ct);
            const float* d = node(nd);
            std::vector<std::pair<float, int>> inner;
            for (int c = 0; c < 4; ++c) {
                if (lk[c] < 0) continue;
                const float blo[3] = {d[c], d[4 + c], d[8 + c]}, bhi[3] = {d[12 + c], d[16 + c], d[20 + c]};
                float tn;
                if (!hit_box(r, blo, bhi, best, tn)) continue;
                if (ct[c] > 0) {
                    for (int m = 0; m < ct[c]; ++m) {
                        const float* t = &H.tris[12 * (size_t)(lk[c] + m)];
                        int32_t id;
                        std::memcpy(&id, t + 3, 4);
                        float tt = hit_tri(r, t, best * 1.0000001f);
                        if (better(tt, id, best, prim)) best = tt, prim = id;
                    }
                } else {
                    inner.push_back({tn, lk[c]});
                }
            }
            inner.erase(std::remove_if(inner.begin(), inner.end(), [&](const std::pair<float, int>& x) {
                            return !(x.first < best);
                        }), inner.end());
            std::sort(inner.begin(), inner.end());
            if (inner.empty()) {
                if (stack.empty()) break;
                nd = stack.back();
                stack.pop_back();
                continue;
            }
            for (size_t j = inner.size() - 1; j >= 1; --j) stack.push_back(inner[j].second);
            max_stack = std::max(max_stack, (int)stack.size());
            nd = inner[0].second;
        }
        hits += bp >= 0;
        differing += bp != prim || (bp >= 0 && bt != best);
    }
    printf("nodes=%d stack_need=%d box_violations=%ld unseen=%ld orphans=%ld rays=%d hits=%ld differing=%ld "
           "max_stack=%d\n",
           H.n_nodes, H.stack_need, bad, unseen, orphans, nr, hits, differing, max_stack);
    return 0;
}
